// lre_batch.hip -- batched estimation (lre_batch_* in include/lre.h): many independent
// instances of steps (i) and (ii) in one persistent kernel driven by a work list.
//
// An instance of at most 7 qubits is one counts-pass tile: one work item runs it from
// the counts to rho inside one workgroup (the phases ordered by workgroup barriers).
// A larger instance is cut into items per stage -- counts-pass tiles, the row-total
// check, the later fold pass, step (ii) per group of x_hi row patterns --
// the same per-block device functions the single-instance kernels run
// (lre_kernels.hpp).  The host lists the items so that an item only ever depends on
// items listed before it.  Each persistent workgroup takes the next item (one atomic
// counter), waits until the items it depends on have finished (per-instance, per-stage
// completion counters, agent-scope acquire), runs it and, when a later item consumes
// its output, releases it and bumps its stage's counter.  Items are taken in list
// order by running workgroups, so every item waited for has already been taken by a
// running workgroup and every wait ends; the wait is bounded anyway (FLAG_WAIT) so
// that no wave can spin forever.  In the staged form the list stops after the counts
// pass and two kernels of their own run the later folds and step (ii) (see
// batch_fold_kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "lre.h"
#include "lre_internal.hpp"
#include "lre_kernels.hpp"

using namespace lre;
using lre_detail::aligned;
using lre_detail::DeviceGuard;

namespace {

constexpr int kBT = 432;          // threads of a persistent workgroup (27 row groups of 16 lanes)
constexpr int kQ = 7;             // counts-pass tile qubits (n >= 7)
constexpr int kJ = 6;             // low step-(ii) qubits (n > 6)
constexpr uint32_t kWaitLimit = 1u << 24;  // sleeps of ~64 clocks before a wait gives up

enum Kind : uint8_t { K_SMALL = 0, K_COUNTS = 1, K_TOTALS = 2, K_FOLD = 3, K_RHO = 4 };
// variant bits (V_PB: the instance has per-basis totals, binary64 sums)
enum : uint8_t { V_MAD24 = 16, V_FP32 = 32, V_RHO = 64, V_PB = 128 };

struct BItem {
  int32_t inst;
  uint8_t kind, variant, pad0, pad1;
  int32_t wait_ctr;      // completion counter to wait for (-1: none)
  uint32_t wait_target;  // value it must reach
  int32_t done_ctr;      // counter to increment when done (-1: none)
  int32_t pad2;
  int64_t begin, end;    // block / column / basis / element range
};

struct BInst {
  const uint16_t* counts;
  double* coef;
  void* rho;
  const uint32_t* nb_in;      // caller's per-basis totals (per-basis mode) or NULL
  uint64_t shots;             // 0: per-basis totals
  int64_t off_part;           // workspace offset of the later-pass partials
  int64_t off_nb, off_inv;    // per-basis mode: N_b and 1/N_b in the workspace
  int32_t n, q1;
};

// Pointers read from the instance table are retyped into the global address space
// (the compiler cannot infer it for pointers loaded from memory and would otherwise use
// flat loads, which also count against the LDS wait counter and turn every wait in the
// prefetching loops into a full wait).
#define LRE_GLOBAL __attribute__((address_space(1)))
// The workgroup's LDS buffer is handed to the (not inlined) item functions typed in the
// LDS address space: as a generic pointer it compiled to a flat-to-LDS conversion with a
// null check before every LDS access of the counts pass.
#define LRE_LDS __attribute__((address_space(3)))

struct BInstG {
  const LRE_GLOBAL uint16_t* counts;
  LRE_GLOBAL double* coef;
  LRE_GLOBAL char* rho;
  uint64_t shots;
  int64_t off_part;
  int32_t n, q1;
};

// The per-basis fields, apart, so that the view every item takes (and the stack frame of
// the uniform-shot item functions) stays small.
struct BInstPB {
  const LRE_GLOBAL uint32_t* nb_in;
  int64_t off_nb, off_inv;
};

__device__ __forceinline__ BInstG global_view(const BInst& I) {
  BInstG G;
  G.counts = (const LRE_GLOBAL uint16_t*)I.counts;
  G.coef = (LRE_GLOBAL double*)I.coef;
  G.rho = (LRE_GLOBAL char*)I.rho;
  G.shots = I.shots;
  G.off_part = I.off_part;
  G.n = I.n;
  G.q1 = I.q1;
  return G;
}

__device__ __forceinline__ BInstPB pb_view(const BInst& I) {
  BInstPB X;
  X.nb_in = (const LRE_GLOBAL uint32_t*)I.nb_in;
  X.off_nb = I.off_nb;
  X.off_inv = I.off_inv;
  return X;
}

constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kLdsCounts = (size_t)StreamGeom<kQ>::NACC * 4 + (size_t)StreamGeom<kQ>::NROWS * 4;
constexpr size_t kLdsRhoLow = 2 * (size_t)RhoLowLds<kJ>::SIZE * 8;
constexpr size_t kLds = cmax(kLdsCounts, kLdsRhoLow);
static_assert(RhoTileGeom<3>::NV * sizeof(double) <= kLds, "step-(ii) units of n = 9 fit the LDS buffer");
// per-basis plans: binary64 accumulators (one workgroup per CU)
constexpr size_t kLdsCountsPB = (size_t)StreamGeom<kQ>::NACC * 8 + (size_t)StreamGeom<kQ>::NROWS * 4;
constexpr size_t kLdsPB = cmax(kLdsCountsPB, kLdsRhoLow);

// The callees below take the instance with global-typed pointers; the generic pointers
// they hand to the shared device functions are casts of them, from which the compiler
// infers global loads and stores.
__device__ __forceinline__ char* g2p(LRE_GLOBAL char* p) { return (char*)p; }
template <typename T>
__device__ __forceinline__ T* l2p(LRE_LDS char* p) { return (T*)p; }

// An instance with n <= 7 (one counts-pass tile) from counts to rho in one workgroup;
// __syncthreads orders the phases (it is a workgroup-scope release/acquire).
template <int Q, typename OutT>
__device__ __forceinline__ void small_rho(const BInstG& I, int tid, double* re, double* im) {
  const double* coef = (const double*)I.coef;
  if constexpr (Q <= kJ) {
    rho_low_block<Q, true, OutT, kBT>(coef, (void*)g2p(I.rho), I.n, 0, tid, re, im);
  } else {
    rho_tiles<Q - kJ, OutT, kBT>(coef, (void*)g2p(I.rho), 0, (int64_t)8 << (Q - kJ), tid, re);
  }
}

template <int Q, bool MAD24, bool PREFETCH>
__device__ __noinline__ void run_small(const BInstG& I, uint8_t var, int tid, LRE_LDS char* smem,
                                       uint32_t* flags) {
  uint32_t* acc = l2p<uint32_t>(smem);
  uint32_t* rs = acc + StreamGeom<Q>::NACC;
  counts_block<Q, kBT, uint32_t, false, Out::CoefUniform, MAD24, PREFETCH>(
      (const uint16_t*)I.counts, I.n, 1, nullptr, (void*)(double*)I.coef, nullptr, I.shots, 0, tid, acc, rs, flags);
  __syncthreads();
  if (var & V_RHO) {
    double* re = l2p<double>(smem);
    double* im = re + (kLds / 16);
    if (var & V_FP32) small_rho<Q, float>(I, tid, re, im);
    else small_rho<Q, double>(I, tid, re, im);
  }
}

// Per-basis totals of bases [b0, b1) (Sec. II eq. 3 frequencies p = c / N_b): N_b, the
// caller's or else the row sum, into the workspace, 1/N_b (correctly rounded) beside
// it, FLAG_EMPTY for an empty basis.  A group of 16 lanes per basis row.
__device__ __noinline__ void run_totals(const BInstG& I, const BInstPB& X, int64_t b0, int64_t b1, int tid,
                                        LRE_GLOBAL char* ws, uint32_t* flags) {
  LRE_GLOBAL uint32_t* nb = (LRE_GLOBAL uint32_t*)(ws + X.off_nb);
  LRE_GLOBAL double* inv = (LRE_GLOBAL double*)(ws + X.off_inv);
  constexpr int kGroups = kBT / 16;
  const int grp = tid / 16, lam = tid % 16;
  const int64_t d = (int64_t)1 << I.n;
  auto put = [&](int64_t b, uint32_t N) __attribute__((always_inline)) {
    if (lam == 0) {
      nb[b] = N;
      inv[b] = N ? 1.0 / (double)N : 0.0;
      if (!N) atomicOr(flags, (uint32_t)FLAG_EMPTY);
    }
  };
  if (X.nb_in) {
    for (int64_t b = b0 + grp; b < b1; b += kGroups) put(b, X.nb_in[b]);
    return;
  }
  if (I.n < 3) {
    for (int64_t b = b0 + grp; b < b1; b += kGroups) {   // uniform within a group
      uint32_t sum = 0;
      for (int64_t o = lam; o < d; o += 16) sum += I.counts[b * d + o];
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 16);
      put(b, sum);
    }
    return;
  }
  // Rows of 2^n >= 8 counts start 16-byte aligned: 16-byte loads of 8 counts, kR rows
  // per group at a time with all their loads issued before any is summed (a row of
  // 2^n <= 512 counts is at most 4 loads per lane).
  typedef uint32_t u32x4_v __attribute__((ext_vector_type(4)));
  constexpr int kW = (1 << LRE_BATCH_MAX_QUBITS) / 8 / 16, kR = 4;
  const int64_t words = d / 8;
  auto hsum = [](const u32x4_v& v) __attribute__((always_inline)) {
    return (v.x & 0xFFFFu) + (v.x >> 16) + (v.y & 0xFFFFu) + (v.y >> 16) + (v.z & 0xFFFFu) + (v.z >> 16) +
           (v.w & 0xFFFFu) + (v.w >> 16);
  };
  for (int64_t b = b0 + grp; b < b1; b += kR * kGroups) {   // uniform within a group
    u32x4_v w[kR][kW];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int64_t br = b + (int64_t)r * kGroups;
      const LRE_GLOBAL u32x4_v* row = (const LRE_GLOBAL u32x4_v*)(I.counts + br * d);
#pragma unroll
      for (int k = 0; k < kW; ++k) {
        const int64_t o = lam + 16 * k;
        w[r][k] = (br < b1 && o < words) ? row[o] : u32x4_v{0u, 0u, 0u, 0u};
      }
    }
    uint32_t sum[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      sum[r] = 0;
#pragma unroll
      for (int k = 0; k < kW; ++k) sum[r] += hsum(w[r][k]);
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) sum[r] += __shfl_xor(sum[r], o, 16);
    }
#pragma unroll
    for (int r = 0; r < kR; ++r)
      if (b + (int64_t)r * kGroups < b1) put(b + (int64_t)r * kGroups, sum[r]);
  }
}

// A per-basis instance with n <= 7 in one workgroup: totals, counts pass with binary64
// accumulators (row totals checked against N_b), step (ii).
template <int Q, bool PREFETCH>
__device__ __noinline__ void run_small_pb(const BInstG& I, const BInstPB& X, uint8_t var, int tid, LRE_GLOBAL char* ws,
                                          LRE_LDS char* smem, uint32_t* flags) {
  run_totals(I, X, 0, ipow3(I.n), tid, ws, flags);
  __syncthreads();  // workgroup scope: the totals written above are visible to the block
  double* acc = l2p<double>(smem);
  uint32_t* rs = reinterpret_cast<uint32_t*>(acc + StreamGeom<Q>::NACC);
  counts_block<Q, kBT, double, true, Out::CoefPerBasis, false, PREFETCH>(
      (const uint16_t*)I.counts, I.n, 1, (const double*)g2p(ws + X.off_inv), (void*)(double*)I.coef, nullptr, 0, 0,
      tid, acc, rs, flags, (const uint32_t*)g2p(ws + X.off_nb));
  __syncthreads();
  if (var & V_RHO) {
    double* re = l2p<double>(smem);
    double* im = re + (kLds / 16);
    if (var & V_FP32) small_rho<Q, float>(I, tid, re, im);
    else small_rho<Q, double>(I, tid, re, im);
  }
}

// Per-basis counts-pass row groups [g0, g1): binary64 partials, rows checked against N_b.
template <bool PREFETCH>
__device__ __noinline__ void run_counts_pb(const BInstG& I, const BInstPB& X, int64_t g0, int64_t g1, int tid,
                                           LRE_GLOBAL char* ws, LRE_LDS char* smem, uint32_t* flags) {
  double* acc = l2p<double>(smem);
  uint32_t* rs = reinterpret_cast<uint32_t*>(acc + StreamGeom<kQ>::NACC);
  void* part = (void*)g2p(ws + I.off_part);
  const double* inv = (const double*)g2p(ws + X.off_inv);
  const uint32_t* nb = (const uint32_t*)g2p(ws + X.off_nb);
  const uint16_t* counts = (const uint16_t*)I.counts;
  const int chunks = 1 << (I.n - kQ);
  for (int64_t g = g0; g < g1; ++g) {
    counts_block<kQ, kBT, double, true, Out::Partial, false, PREFETCH>(counts, I.n, chunks, inv, part, nullptr, 0, g,
                                                                      tid, acc, rs, flags, nb);
    __syncthreads();
  }
}

// Row groups [g0, g1) (3^7 rows each): one block call per group covering all 2^(n-7)
// outcome tiles of its rows, so the row totals are complete and checked in the block.
template <bool MAD24, bool PREFETCH>
__device__ __noinline__ void run_counts(const BInstG& I, int64_t g0, int64_t g1, int tid, LRE_GLOBAL char* ws,
                                        LRE_LDS char* smem, uint32_t* flags) {
  uint32_t* acc = l2p<uint32_t>(smem);
  uint32_t* rs = acc + StreamGeom<kQ>::NACC;
  void* part = (void*)g2p(ws + I.off_part);
  const uint16_t* counts = (const uint16_t*)I.counts;
  const int chunks = 1 << (I.n - kQ);
  for (int64_t g = g0; g < g1; ++g) {
    counts_block<kQ, kBT, uint32_t, false, Out::Partial, MAD24, PREFETCH>(counts, I.n, chunks, nullptr, part, nullptr,
                                                                         I.shots, g, tid, acc, rs, flags);
    __syncthreads();  // the next group clears the LDS this one still reads
  }
}

// Final fold of F = n - 7 qubits over columns [c0, c1): every thread first gathers the
// 6^F inputs of C columns into registers, then folds them.  (Folding straight from
// memory serialises the columns: the next column's loads cannot pass this column's
// coefficient stores, and the loads' wait covers the stores.)
template <int F, typename Tin, Out MODE>
__device__ __forceinline__ void fold_cols(const Tin* in, double* coef, int n, uint64_t shots, int64_t c0,
                                          int64_t c1, int tid) {
  constexpr int NIN = (int)ipow3(F) << F, C = 4;
  for (int64_t base = c0 + tid; base < c1; base += (int64_t)kBT * C) {
    Tin x[C][NIN];
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int64_t col = base + (int64_t)j * kBT;
      if (col < c1) {
#pragma unroll
        for (int beta = 0; beta < (int)ipow3(F); ++beta)
#pragma unroll
          for (int sg = 0; sg < (1 << F); ++sg) x[j][beta * (1 << F) + sg] = in[fold_in_offset<F>(F, kQ, col, beta, sg)];
      }
    }
#pragma unroll
    for (int j = 0; j < C; ++j) {
      const int64_t col = base + (int64_t)j * kBT;
      if (col < c1)
        fold_partial_col_src<F, Tin, Tin, MODE>(
            [&](int beta, int sg) __attribute__((always_inline)) { return x[j][beta * (1 << F) + sg]; }, coef,
            n, F, kQ, shots, col);
    }
  }
}

__device__ __noinline__ void run_fold(const BInstG& I, int64_t c0, int64_t c1, int tid, LRE_GLOBAL char* ws) {
  const uint32_t* in = reinterpret_cast<const uint32_t*>(g2p(ws + I.off_part));
  double* coef = (double*)I.coef;
  const int h = I.n - kQ;
  if (h == 1) fold_cols<1, uint32_t, Out::CoefUniform>(in, coef, I.n, I.shots, c0, c1, tid);
  else fold_cols<2, uint32_t, Out::CoefUniform>(in, coef, I.n, I.shots, c0, c1, tid);
}

__device__ __noinline__ void run_fold_pb(const BInstG& I, int64_t c0, int64_t c1, int tid, LRE_GLOBAL char* ws) {
  const double* in = reinterpret_cast<const double*>(g2p(ws + I.off_part));
  double* coef = (double*)I.coef;
  const int h = I.n - kQ;
  if (h == 1) fold_cols<1, double, Out::CoefPerBasis>(in, coef, I.n, 0, c0, c1, tid);
  else fold_cols<2, double, Out::CoefPerBasis>(in, coef, I.n, 0, c0, c1, tid);
}

// Step (ii) for the high patterns x_hi in [x0, x1) of an instance with n = 8 or 9: the
// units (x_hi, xb) of those patterns in sequence, each from coefficients to mu inside
// this workgroup (no intermediate in device memory).
template <typename OutT>
__device__ __noinline__ void run_rho(const BInstG& I, int64_t x0, int64_t x1, int tid, LRE_LDS char* smem) {
  double* V = l2p<double>(smem);
  const double* coef = (const double*)I.coef;
  void* rho = (void*)g2p(I.rho);
  if (I.n == kJ + 2) rho_tiles<2, OutT, kBT>(coef, rho, x0 * 8, x1 * 8, tid, V);
  else rho_tiles<3, OutT, kBT>(coef, rho, x0 * 8, x1 * 8, tid, V);
}

template <bool PREFETCH>
__device__ __forceinline__ void dispatch_small(const BInstG& I, uint8_t var, int tid, LRE_LDS char* smem,
                                               uint32_t* flags) {
  switch (I.n) {
    case 1: run_small<1, false, PREFETCH>(I, var, tid, smem, flags); break;
    case 2: run_small<2, false, PREFETCH>(I, var, tid, smem, flags); break;
    case 3: run_small<3, false, PREFETCH>(I, var, tid, smem, flags); break;
    case 4: run_small<4, false, PREFETCH>(I, var, tid, smem, flags); break;
    case 5: run_small<5, false, PREFETCH>(I, var, tid, smem, flags); break;
    case 6: run_small<6, false, PREFETCH>(I, var, tid, smem, flags); break;
    default:
      if (var & V_MAD24) run_small<7, true, PREFETCH>(I, var, tid, smem, flags);
      else run_small<7, false, PREFETCH>(I, var, tid, smem, flags);
      break;
  }
}

template <bool PREFETCH>
__device__ __forceinline__ void dispatch_small_pb(const BInstG& I, const BInstPB& X, uint8_t var, int tid,
                                                  LRE_GLOBAL char* ws, LRE_LDS char* smem, uint32_t* flags) {
  switch (I.n) {
    case 1: run_small_pb<1, PREFETCH>(I, X, var, tid, ws, smem, flags); break;
    case 2: run_small_pb<2, PREFETCH>(I, X, var, tid, ws, smem, flags); break;
    case 3: run_small_pb<3, PREFETCH>(I, X, var, tid, ws, smem, flags); break;
    case 4: run_small_pb<4, PREFETCH>(I, X, var, tid, ws, smem, flags); break;
    case 5: run_small_pb<5, PREFETCH>(I, X, var, tid, ws, smem, flags); break;
    case 6: run_small_pb<6, PREFETCH>(I, X, var, tid, ws, smem, flags); break;
    default: run_small_pb<7, PREFETCH>(I, X, var, tid, ws, smem, flags); break;
  }
}

// ctl[0]: next item; ctl[1 + 3 j + k]: completion counter of instance j's counts pass
// (k = 0), later fold (k = 1) and per-basis totals (k = 2).
// WORKERS: persistent workgroups per CU the launch is shaped for (one: registers for the
// row prefetch; two: no prefetch, 128 registers).  PB: the plan has per-basis instances
// (binary64 counts-pass accumulators, one workgroup per CU); only then are their item
// variants compiled in.
template <int WORKERS, bool PB>
__global__ __launch_bounds__(kBT, WORKERS == 2 ? 4 : 1) void batch_kernel(
    const BItem* __restrict__ items, const int* __restrict__ nitems_ptr, const BInst* __restrict__ insts,
    char* __restrict__ ws_arg, uint32_t* __restrict__ ctl, uint32_t* __restrict__ flags) {
  constexpr bool PF = WORKERS == 1;
  static_assert(!PB || WORKERS == 1, "per-basis plans run one workgroup per CU");
  __shared__ __align__(16) char smem_arr[PB ? kLdsPB : kLds];
  LRE_LDS char* smem = (LRE_LDS char*)smem_arr;
  __shared__ int s_item;
  __shared__ int s_skip;
  const int tid = threadIdx.x;
  LRE_GLOBAL char* ws = (LRE_GLOBAL char*)ws_arg;
  // The item count lives beside the list (not in the launch arguments), so a launch
  // captured into a graph runs whatever list the plan holds when it is replayed.
  const int nitems = *nitems_ptr;
  for (;;) {
    if (tid == 0) s_item = (int)atomicAdd(&ctl[0], 1u);
    __syncthreads();
    const int it = s_item;
    if (it >= nitems) break;
    const BItem W = items[it];
    if (W.wait_ctr >= 0) {
      if (tid == 0) {
        int skip = 0;
        uint32_t spins = 0;
        while (__hip_atomic_load(&ctl[W.wait_ctr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < W.wait_target) {
          if (++spins > kWaitLimit) {
            atomicOr(flags, (uint32_t)FLAG_WAIT);
            skip = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        s_skip = skip;
      }
      __syncthreads();
      // Acquire: the producers' results become visible to every thread of this workgroup.
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (s_skip) continue;  // uniform: the skipped item's counter never moves, its consumers time out too
    }
    const BInstG I = global_view(insts[W.inst]);
    const bool pb = PB && (W.variant & V_PB);
    switch (W.kind) {
      case K_SMALL:
        if constexpr (PB) {
          if (pb) {
            dispatch_small_pb<PF>(I, pb_view(insts[W.inst]), W.variant, tid, ws, smem, flags);
            break;
          }
        }
        dispatch_small<PF>(I, W.variant, tid, smem, flags);
        break;
      case K_COUNTS:
        if constexpr (PB) {
          if (pb) {
            run_counts_pb<PF>(I, pb_view(insts[W.inst]), W.begin, W.end, tid, ws, smem, flags);
            break;
          }
        }
        if (W.variant & V_MAD24) run_counts<true, PF>(I, W.begin, W.end, tid, ws, smem, flags);
        else run_counts<false, PF>(I, W.begin, W.end, tid, ws, smem, flags);
        break;
      case K_TOTALS:
        if constexpr (PB) run_totals(I, pb_view(insts[W.inst]), W.begin, W.end, tid, ws, flags);
        break;
      case K_FOLD:
        if constexpr (PB) {
          if (pb) {
            run_fold_pb(I, W.begin, W.end, tid, ws);
            break;
          }
        }
        run_fold(I, W.begin, W.end, tid, ws);
        break;
      default:
        if (W.variant & V_FP32) run_rho<float>(I, W.begin, W.end, tid, smem);
        else run_rho<double>(I, W.begin, W.end, tid, smem);
        break;
    }
    if (W.done_ctr >= 0) {
      // Release: this workgroup's results are visible device-wide before the counter moves.
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __syncthreads();
      if (tid == 0) __hip_atomic_fetch_add(&ctl[W.done_ctr], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      __syncthreads();  // s_item and the LDS are reused by the next item
    }
  }
}

// Staged form (lre_batch_tiles.staged = 1): the work list holds only the per-basis
// totals, the counts pass and the instances of at most 7 qubits (those of exactly 7
// without their step (ii)); the later fold and step (ii) run afterwards, in stream
// order, as the two kernels below, shaped for their own work (many small workgroups instead of one 7-wave worker
// per CU).  Both read the plan's form from device memory (stage[1]) and do nothing for
// an unstaged list, so that a captured launch stays valid whichever shape the plan
// takes later.  Blocks are persistent (the grid is fixed when the plan is made) and
// walk their work with a stride of the grid.

// The later fold of every instance with n > 7: 4^7 columns per instance, 256 per block
// (64 blocks per instance), one thread per column, the fold items' column function.
template <bool PB>
__global__ __launch_bounds__(256) void batch_fold_kernel(const int* __restrict__ stage,
                                                         const int32_t* __restrict__ fold_inst, int nblocks,
                                                         const BInst* __restrict__ insts, char* __restrict__ ws_arg) {
  if (stage[1] == 0) return;
  LRE_GLOBAL char* ws = (LRE_GLOBAL char*)ws_arg;
  for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
    const BInst& D = insts[fold_inst[b]];   // 64 consecutive blocks per instance
    const BInstG I = global_view(D);
    const int64_t col = ((int64_t)(b & 63) << 8) | threadIdx.x;
    double* coef = (double*)I.coef;
    const int F = I.n - kQ;
    if (PB && I.shots == 0) {
      const double* in = reinterpret_cast<const double*>(g2p(ws + I.off_part));
      if (F == 1) fold_partial_col<1, double, double, Out::CoefPerBasis>(in, coef, I.n, 1, kQ, 0, col);
      else fold_partial_col<2, double, double, Out::CoefPerBasis>(in, coef, I.n, 2, kQ, 0, col);
    } else {
      const uint32_t* in = reinterpret_cast<const uint32_t*>(g2p(ws + I.off_part));
      if (F == 1) fold_partial_col<1, uint32_t, uint32_t, Out::CoefUniform>(in, coef, I.n, 1, kQ, I.shots, col);
      else fold_partial_col<2, uint32_t, uint32_t, Out::CoefUniform>(in, coef, I.n, 2, kQ, I.shots, col);
    }
  }
}

// Step (ii) of every instance with n >= 7: one rho_tiles unit (x_hi, 8 x_lo) per block.
template <typename OutT>
__global__ __launch_bounds__(256) void batch_rho_kernel(const int* __restrict__ stage, const int2* __restrict__ units,
                                                        int nblocks, const BInst* __restrict__ insts) {
  __shared__ double V[RhoTileGeom<3>::NV];
  if (stage[1] == 0) return;
  for (int b = blockIdx.x; b < nblocks; b += gridDim.x) {
    const int2 w = units[b];
    const BInstG I = global_view(insts[w.x]);
    const double* coef = (const double*)I.coef;
    void* rho = (void*)g2p(I.rho);
    if (I.n == kJ + 1) rho_tiles<1, OutT, 256>(coef, rho, w.y, (int64_t)w.y + 1, threadIdx.x, V);
    else if (I.n == kJ + 2) rho_tiles<2, OutT, 256>(coef, rho, w.y, (int64_t)w.y + 1, threadIdx.x, V);
    else rho_tiles<3, OutT, 256>(coef, rho, w.y, (int64_t)w.y + 1, threadIdx.x, V);
    lds_barrier();  // the next unit's staging overwrites V
  }
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct InstMeta {
  int n = 0, q1 = 0, F = 0;     // F: later-pass qubits (n - 7 when n > 7)
  int64_t blocks1 = 0;          // counts-pass tiles
  bool mad24 = false;
  bool pb = false;              // per-basis totals
  int64_t counts = 0;           // 6^n, the ordering key
};

}  // namespace

struct lre_batch {
  lre_ctx* ctx = nullptr;
  uint32_t flags = 0;
  std::vector<lre_instance> inst;
  std::vector<InstMeta> meta;
  std::vector<BInst> dinst_host;
  lre_batch_tiles tiles{};
  BInst* d_inst = nullptr;
  BItem* d_items = nullptr;     // work list, allocated once at the largest list any
  int* d_nitems = nullptr;      // shape can give (fixed addresses for captured runs);
                                // [0] item count, [1] staged form
  int32_t* d_fold = nullptr;    // staged form: instance of each fold block (64 per
  int2* d_units = nullptr;      // instance of n > 7) and (instance, unit) of each rho block
  int nfold = 0, nunits = 0;
  size_t items_cap = 0;
  int nitems = 0;
  size_t ctl_bytes = 0;
  size_t ws_bytes = 0;
  int num_cu = 0;
  bool pb = false;              // some instance has per-basis totals
};

namespace {

bool valid_tiles(const lre_batch_tiles& t) {
  return (t.workers_per_cu == 1 || t.workers_per_cu == 2) && t.counts_tiles >= 1 && t.fold_cols >= kBT &&
         t.fold_cols % kBT == 0 && t.rho_blocks >= 1 && (t.interleave == 0 || t.interleave == 1) &&
         (t.staged == 0 || t.staged == 1);
}

void add_range(std::vector<BItem>& out, int inst, Kind kind, uint8_t var, int64_t total, int64_t per,
               int32_t wait_ctr, uint32_t wait_target, int32_t done_ctr, uint32_t* count_out) {
  // ceil(total / per) items of equal size (to one unit): an uneven last item would
  // finish long after its siblings and hold up the stage that waits for all of them
  const int64_t parts = (total + per - 1) / per;
  uint32_t c = 0;
  for (int64_t k = 0; k < parts; ++k) {
    BItem W{};
    W.inst = inst;
    W.kind = kind;
    W.variant = var;
    W.wait_ctr = wait_ctr;
    W.wait_target = wait_target;
    W.done_ctr = done_ctr;
    W.begin = total * k / parts;
    W.end = total * (k + 1) / parts;
    out.push_back(W);
    ++c;
  }
  if (count_out) *count_out = c;
}

// Work items of instance j for one stage (0 per-basis totals, 1 counts, 2 check + fold,
// 3 rho).
struct StageCounts {
  uint32_t totals = 0, counts = 0, fold = 0;
};

constexpr int kStages = 4;
constexpr int64_t kTotalsPerItem = 2048;  // bases per per-basis totals item

void emit_stage(const lre_batch& B, const lre_batch_tiles& t, int j, int stage, std::vector<BItem>& out,
                StageCounts& sc) {
  const InstMeta& m = B.meta[j];
  const bool want_rho = !(B.flags & LRE_NO_RHO);
  const uint8_t fp32 = (B.flags & LRE_RHO_FP32) ? V_FP32 : 0;
  const uint8_t mad = m.mad24 ? V_MAD24 : 0;
  const uint8_t pb = m.pb ? V_PB : 0;
  const int32_t c_counts = 1 + 3 * j, c_fold = 2 + 3 * j, c_tot = 3 + 3 * j;
  if (m.n <= kQ) {  // one tile: the whole instance is one item
    // (staged: step (ii) of a 7-qubit instance runs in the step-(ii) kernel instead)
    const bool rho_here = want_rho && !(t.staged && m.n == kQ);
    if (stage == 0)
      add_range(out, j, K_SMALL, (uint8_t)(mad | fp32 | pb | (rho_here ? V_RHO : 0)), 1, 1, -1, 0, -1, nullptr);
    return;
  }
  switch (stage) {
    case 0:  // per-basis totals and their reciprocals
      if (m.pb) add_range(out, j, K_TOTALS, pb, ipow3(m.n), kTotalsPerItem, -1, 0, c_tot, &sc.totals);
      break;
    case 1:  // row groups of 3^7 bases, each with all its outcome tiles
      add_range(out, j, K_COUNTS, (uint8_t)(mad | pb), ipow3(m.n - kQ), t.counts_tiles, m.pb ? c_tot : -1,
                sc.totals, c_counts, &sc.counts);
      break;
    case 2:
      add_range(out, j, K_FOLD, pb, ipow4(kQ), t.fold_cols, c_counts, sc.counts, want_rho ? c_fold : -1, &sc.fold);
      break;
    case 3:
      if (want_rho)
        add_range(out, j, K_RHO, fp32, (int64_t)1 << (m.n - kJ), t.rho_blocks, c_fold, sc.fold, -1, nullptr);
      break;
    default:
      break;
  }
}

// The work list of the plan's instances under work-item shape t.
std::vector<BItem> list_items(const lre_batch& B, const lre_batch_tiles& t) {
  const int count = (int)B.inst.size();
  std::vector<int> order(count);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return B.meta[a].counts > B.meta[b].counts; });
  std::vector<BItem> items;
  std::vector<StageCounts> sc(count);
  const int stages = t.staged ? 2 : kStages;   // staged: folds and step (ii) run as kernels of their own
  if (t.interleave) {
    for (int j : order)
      for (int s = 0; s < stages; ++s) emit_stage(B, t, j, s, items, sc[j]);
  } else if (t.staged) {
    // the long counts-pass items first, the one-item instances (n <= 7) after them to
    // fill the end of the launch, largest first
    for (int s = 0; s < stages; ++s)
      for (int j : order)
        if (B.meta[j].n > kQ) emit_stage(B, t, j, s, items, sc[j]);
    for (int j : order)
      if (B.meta[j].n <= kQ) emit_stage(B, t, j, 0, items, sc[j]);
  } else {
    for (int s = 0; s < stages; ++s)
      for (int j : order) emit_stage(B, t, j, s, items, sc[j]);
  }
  return items;
}

// Upload the list of the plan's current shape into the fixed device list.
lre_status rebuild(lre_batch& B) {
  const std::vector<BItem> items = list_items(B, B.tiles);
  if (items.size() > B.items_cap) return LRE_E_UNSUPPORTED;  // the capacity is the largest list
  DeviceGuard g(B.ctx->device);
  if (!g.ok) return LRE_E_HIP;
  // A run still in flight may read the current list: wait before replacing it.
  if (hipDeviceSynchronize() != hipSuccess) return LRE_E_HIP;
  if (!items.empty() &&
      hipMemcpy(B.d_items, items.data(), items.size() * sizeof(BItem), hipMemcpyHostToDevice) != hipSuccess)
    return LRE_E_HIP;
  const int hdr[2] = {(int)items.size(), B.tiles.staged};
  if (hipMemcpy(B.d_nitems, hdr, sizeof hdr, hipMemcpyHostToDevice) != hipSuccess) return LRE_E_HIP;
  const int cnt = hdr[0];
  B.nitems = cnt;
  return LRE_OK;
}

// The staged form's fold and step-(ii) kernels (they return at once for an unstaged
// list; see batch_fold_kernel).
void launch_staged(const lre_batch& B, char* ws, hipStream_t st) {
  if (B.nfold) {
    const unsigned grid = (unsigned)std::min(B.nfold, B.num_cu * 8);
    if (B.pb)
      hipLaunchKernelGGL((batch_fold_kernel<true>), dim3(grid), dim3(256), 0, st, (const int*)B.d_nitems,
                         (const int32_t*)B.d_fold, B.nfold, (const BInst*)B.d_inst, ws);
    else
      hipLaunchKernelGGL((batch_fold_kernel<false>), dim3(grid), dim3(256), 0, st, (const int*)B.d_nitems,
                         (const int32_t*)B.d_fold, B.nfold, (const BInst*)B.d_inst, ws);
  }
  if (B.nunits) {
    const unsigned grid = (unsigned)std::min(B.nunits, B.num_cu * 4);
    if (B.flags & LRE_RHO_FP32)
      hipLaunchKernelGGL((batch_rho_kernel<float>), dim3(grid), dim3(256), 0, st, (const int*)B.d_nitems,
                         (const int2*)B.d_units, B.nunits, (const BInst*)B.d_inst);
    else
      hipLaunchKernelGGL((batch_rho_kernel<double>), dim3(grid), dim3(256), 0, st, (const int*)B.d_nitems,
                         (const int2*)B.d_units, B.nunits, (const BInst*)B.d_inst);
  }
}

}  // namespace

extern "C" {

lre_status lre_batch_plan(lre_ctx* ctx, const lre_instance* inst, int count, uint32_t flags,
                          lre_batch** plan_out) {
  if (!plan_out) return LRE_E_ARG;
  *plan_out = nullptr;
  if (!ctx || !inst || count < 1) return LRE_E_ARG;
  if (flags & ~(LRE_NO_RHO | LRE_RHO_FP32)) return LRE_E_ARG;
  const bool want_rho = !(flags & LRE_NO_RHO);
  for (int j = 0; j < count; ++j) {
    const lre_instance& I = inst[j];
    if (I.n < 1 || !I.counts || !I.coef || !aligned(I.counts, 16) || !aligned(I.coef, 8)) return LRE_E_ARG;
    if (I.n > LRE_BATCH_MAX_QUBITS) return LRE_E_UNSUPPORTED;
    if (I.shots == 0 && I.n_per_basis && !aligned(I.n_per_basis, 4)) return LRE_E_ARG;
    if ((long double)I.shots * (long double)ipow3(I.n) > (long double)INT32_MAX) return LRE_E_ARG;
    if (want_rho && (!I.rho || !aligned(I.rho, 16))) return LRE_E_ARG;
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return LRE_E_HIP;
  lre_batch* B = new (std::nothrow) lre_batch;
  if (!B) return LRE_E_HIP;
  B->ctx = ctx;
  B->flags = flags;
  B->inst.assign(inst, inst + count);
  B->meta.resize(count);
  B->dinst_host.resize(count);
  if (hipDeviceGetAttribute(&B->num_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
      B->num_cu < 1) {
    delete B;
    return LRE_E_HIP;
  }
  B->ctl_bytes = align256((size_t)(1 + 3 * (size_t)count) * 4);
  size_t off = B->ctl_bytes;
  for (int j = 0; j < count; ++j) {
    const lre_instance& I = inst[j];
    InstMeta& m = B->meta[j];
    m.n = I.n;
    m.q1 = I.n < kQ ? I.n : kQ;
    m.F = I.n > kQ ? I.n - kQ : 0;
    m.blocks1 = ipow3(I.n - m.q1) << (I.n - m.q1);
    m.pb = I.shots == 0;
    m.mad24 = !m.pb && m.q1 == kQ && 27ull * I.shots < (1ull << 23);
    m.counts = ipow3(I.n) << I.n;
    B->pb = B->pb || m.pb;
    BInst& d = B->dinst_host[j];
    d.counts = I.counts;
    d.coef = I.coef;
    d.rho = I.rho;
    d.nb_in = m.pb ? I.n_per_basis : nullptr;
    d.shots = I.shots;
    d.n = I.n;
    d.q1 = m.q1;
    d.off_part = 0;
    if (m.F > 0) {
      d.off_part = (int64_t)off;
      off += align256((size_t)m.blocks1 * (size_t)ipow4(kQ) * (m.pb ? 8 : 4));
    }
    d.off_nb = d.off_inv = 0;
    if (m.pb) {
      d.off_nb = (int64_t)off;
      off += align256((size_t)ipow3(I.n) * 4);
      d.off_inv = (int64_t)off;
      off += align256((size_t)ipow3(I.n) * 8);
    }
  }
  B->ws_bytes = off;
  if (hipMalloc(&B->d_inst, count * sizeof(BInst)) != hipSuccess) {
    delete B;
    return LRE_E_HIP;
  }
  if (hipMemcpy(B->d_inst, B->dinst_host.data(), count * sizeof(BInst), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(B->d_inst);
    delete B;
    return LRE_E_HIP;
  }
  // The smallest shape (one row group, kBT columns, one row pattern per item) gives
  // the longest list; the list is allocated once at that length.
  const size_t cap = list_items(*B, lre_batch_tiles{1, 1, kBT, 1, 0, 0}).size();
  if (cap > (size_t)INT32_MAX) {
    lre_batch_destroy(B);
    return LRE_E_UNSUPPORTED;
  }
  if (hipMalloc(&B->d_items, std::max<size_t>(cap, 1) * sizeof(BItem)) != hipSuccess ||
      hipMalloc(&B->d_nitems, 256) != hipSuccess) {
    lre_batch_destroy(B);
    return LRE_E_HIP;
  }
  B->items_cap = cap;
  // staged form: fold blocks and step-(ii) units of the instances with n > 7
  std::vector<int32_t> fold;
  std::vector<int2> units;
  for (int j = 0; j < count; ++j) {
    if (B->meta[j].n < kQ) continue;
    if (B->meta[j].n > kQ)
      for (int k = 0; k < 64; ++k) fold.push_back(j);
    if (want_rho)
      for (int u = 0; u < (8 << (B->meta[j].n - kJ)); ++u) units.push_back(make_int2(j, u));
  }
  B->nfold = (int)fold.size();
  B->nunits = (int)units.size();
  if ((B->nfold && hipMalloc(&B->d_fold, fold.size() * sizeof(int32_t)) != hipSuccess) ||
      (B->nunits && hipMalloc(&B->d_units, units.size() * sizeof(int2)) != hipSuccess)) {
    lre_batch_destroy(B);
    return LRE_E_HIP;
  }
  if ((B->nfold && hipMemcpy(B->d_fold, fold.data(), fold.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) ||
      (B->nunits && hipMemcpy(B->d_units, units.data(), units.size() * sizeof(int2), hipMemcpyHostToDevice) != hipSuccess)) {
    lre_batch_destroy(B);
    return LRE_E_HIP;
  }
  B->tiles = lre_batch_tiles{1, 4, kBT * 16, 1, 0, 0};
  const lre_status s = rebuild(*B);
  if (s != LRE_OK) {
    lre_batch_destroy(B);
    return s;
  }
  *plan_out = B;
  return LRE_OK;
}

size_t lre_batch_workspace_bytes(const lre_batch* plan) { return plan ? plan->ws_bytes : 0; }

lre_status lre_batch_set_tiles(lre_batch* plan, const lre_batch_tiles* tiles) {
  if (!plan || !tiles || !valid_tiles(*tiles)) return LRE_E_ARG;
  plan->tiles = *tiles;
  return rebuild(*plan);
}

lre_status lre_batch_get_tiles(const lre_batch* plan, lre_batch_tiles* tiles, int* num_items) {
  if (!plan) return LRE_E_ARG;
  if (tiles) *tiles = plan->tiles;
  if (num_items) *num_items = plan->nitems;
  return LRE_OK;
}

lre_status lre_batch_run(lre_batch* plan, void* workspace, size_t workspace_bytes, void* stream) {
  if (!plan) return LRE_E_ARG;
  if (!workspace || !aligned(workspace, 256)) return LRE_E_ARG;
  if (workspace_bytes < plan->ws_bytes) return LRE_E_WORKSPACE;
  DeviceGuard g(plan->ctx->device);
  if (!g.ok) return LRE_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  uint32_t* ctl = reinterpret_cast<uint32_t*>(ws);
  const int64_t words = 1 + 3 * (int64_t)plan->inst.size();
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, st, ctl, words, 0u);
  if (plan->pb) {  // binary64 accumulators: one workgroup per CU
    hipLaunchKernelGGL((batch_kernel<1, true>), dim3((unsigned)plan->num_cu), dim3(kBT), 0, st,
                       (const BItem*)plan->d_items, (const int*)plan->d_nitems, (const BInst*)plan->d_inst, ws, ctl,
                       plan->ctx->flags);
    launch_staged(*plan, ws, st);
    return hipGetLastError() == hipSuccess ? LRE_OK : LRE_E_HIP;
  }
  const int workers = plan->num_cu * plan->tiles.workers_per_cu;
  if (plan->tiles.workers_per_cu == 1)
    hipLaunchKernelGGL((batch_kernel<1, false>), dim3((unsigned)workers), dim3(kBT), 0, st, (const BItem*)plan->d_items,
                       (const int*)plan->d_nitems, (const BInst*)plan->d_inst, ws, ctl, plan->ctx->flags);
  else
    hipLaunchKernelGGL((batch_kernel<2, false>), dim3((unsigned)workers), dim3(kBT), 0, st, (const BItem*)plan->d_items,
                       (const int*)plan->d_nitems, (const BInst*)plan->d_inst, ws, ctl, plan->ctx->flags);
  launch_staged(*plan, ws, st);
  return hipGetLastError() == hipSuccess ? LRE_OK : LRE_E_HIP;
}

lre_status lre_batch_tune(lre_batch* plan, void* workspace, size_t workspace_bytes, int reps, double* best_ms,
                          void* stream) {
  if (!plan || reps < 1) return LRE_E_ARG;
  DeviceGuard g(plan->ctx->device);
  if (!g.ok) return LRE_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return LRE_E_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return LRE_E_HIP;
  }
  const lre_batch_tiles start = plan->tiles;
  lre_batch_tiles best = start;
  double best_t = 1e300;
  lre_status s = LRE_OK;
  for (int sg : {0, 1})
  for (int w : {1, 2})
    for (int ct : {1, 2, 4, 8, 16})
      for (int fc : {kBT * 4, kBT * 16})
        for (int rb : {1, 2, 4})
          for (int il : {0, 1}) {
            if (w == 2 && plan->pb) continue;  // per-basis plans run one workgroup per CU
            // unstaged: 1, 2 or 4 row groups per counts item; staged: the fold and
            // step-(ii) shapes are those of their own kernels
            if (!sg && ct > 4) continue;
            if (sg && (fc != kBT * 16 || rb != 1 || il != 0)) continue;
            const lre_batch_tiles t{w, ct, fc, rb, il, sg};
            if ((s = lre_batch_set_tiles(plan, &t)) != LRE_OK) goto done;
            if ((s = lre_batch_run(plan, workspace, workspace_bytes, stream)) != LRE_OK) goto done;
            if (hipEventRecord(e0, st) != hipSuccess) { s = LRE_E_HIP; goto done; }
            for (int r = 0; r < reps; ++r)
              if ((s = lre_batch_run(plan, workspace, workspace_bytes, stream)) != LRE_OK) goto done;
            if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
              s = LRE_E_HIP;
              goto done;
            }
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { s = LRE_E_HIP; goto done; }
            const double t_ms = (double)ms / reps;
            if (t_ms < best_t) {
              best_t = t_ms;
              best = t;
            }
          }
done:
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  const lre_status s2 = lre_batch_set_tiles(plan, s == LRE_OK ? &best : &start);
  if (s == LRE_OK) s = s2;
  if (s == LRE_OK && best_ms) *best_ms = best_t;
  return s;
}

void lre_batch_destroy(lre_batch* plan) {
  if (!plan) return;
  {
    DeviceGuard g(plan->ctx->device);
    if (plan->d_items) (void)hipFree(plan->d_items);
    if (plan->d_nitems) (void)hipFree(plan->d_nitems);
    if (plan->d_inst) (void)hipFree(plan->d_inst);
    if (plan->d_fold) (void)hipFree(plan->d_fold);
    if (plan->d_units) (void)hipFree(plan->d_units);
  }
  delete plan;
}

}  // extern "C"
