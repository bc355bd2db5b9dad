// lre_abi.hip -- the C ABI declared in include/lre.h: argument checks, pass planning,
// workspace layout and kernel launches.  All arithmetic runs in lre_kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "lre.h"
#include "lre_internal.hpp"
#include "lre_kernels.hpp"
#include "lre_povm.hpp"

using namespace lre;
using lre_detail::aligned;
using lre_detail::DeviceGuard;
using lre_detail::record_stage;


// Workspace of lre_estimate_noalloc: one copy per device, held until the process
// ends.  Host code never passes this name to a kernel (on the host it is a stand-in,
// not a device address); it uses the per-device address lre_create resolves with
// hipGetSymbolAddress, kept in lre_ctx::scratch.
static __device__ __align__(256) char scratch[LRE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxQ1 = 7;     // qubits folded by the counts pass
constexpr int kMaxF = 3;      // qubits folded by a later pass in registers
constexpr int kMaxFLast = 2;  // qubits folded by the final pass (below kMinHF4)
constexpr int kMinHF4 = 5;    // from this many unfolded qubits on, the first later pass
                              // folds 4 with LDS accumulators and the final one the rest
constexpr int kRhoJ = 6;      // qubits of the low step-(ii) transform
// Step (ii) goes through a complex128 intermediate of 4^n entries only beyond 12 qubits
// (up to 10 the LDS tiles, at 11 and 12 the real-arithmetic tiles need none).
constexpr bool rho_needs_tmp(int n) { return n > kRhoJ + 6; }

enum class Ty : int { U32 = 0, F64 = 1 };

size_t ty_size(Ty t) { return t == Ty::U32 ? 4 : 8; }
size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Plan {
  int n = 0;
  bool per_basis = false;
  int q1 = 0;
  int chunks = 1;            // tiles per counts-pass block
  int64_t blocks1 = 0;       // counts-pass blocks
  Ty t1 = Ty::U32;           // counts-pass accumulator / output type
  int npass = 0;             // later passes
  int F[8] = {0};
  Ty tout[8] = {Ty::U32};
  int J = 0;                 // low step-(ii) qubits
  size_t off_a = 0, off_b = 0, off_rowpart = 0, off_nb = 0, off_inv = 0, off_tmp = 0, total = 0;
};

// Partial sums after folding f qubits are bounded by 3^f * (basis total).
Ty int_type_for(int folded, uint64_t shots) {
  long double bound = (long double)shots;
  for (int i = 0; i < folded; ++i) bound *= 3.0L;
  return bound <= (long double)INT32_MAX ? Ty::U32 : Ty::F64;
}

bool make_plan(int n, uint64_t shots, uint32_t flags, Plan& P) {
  if (n < 1 || n > LRE_MAX_QUBITS) return false;
  P = Plan();
  P.n = n;
  P.per_basis = shots == 0;
  P.q1 = n < kMaxQ1 ? n : kMaxQ1;
  const int64_t tiles_per_row = (int64_t)1 << (n - P.q1);
  const int64_t row_groups = ipow3(n - P.q1);
  int64_t chunks = 1;
  while (chunks * 2 <= tiles_per_row && chunks < 16 &&
         row_groups * (tiles_per_row / (chunks * 2)) >= 1024)
    chunks *= 2;
  P.chunks = (int)chunks;
  P.blocks1 = row_groups * (tiles_per_row / chunks);
  P.t1 = P.per_basis ? Ty::F64 : int_type_for(P.q1, shots);

  // Later passes: the last folds at most kMaxFLast qubits (it also divides every
  // output, which costs registers); the others split the rest evenly, <= kMaxF each.
  const int h = n - P.q1;
  if (h >= kMinHF4 && h <= 4 + kMaxF) {
    // Two passes: 4 qubits (LDS) then the remaining 1..3 in registers, which reads and
    // writes far less than 3 + 2 + 2 (53 GB instead of 70 GB of partials at n = 14).
    P.npass = 2;
    P.F[0] = 4;
    P.F[1] = h - 4;
  } else {
    const int last = h < kMaxFLast ? h : kMaxFLast;
    const int rest = h - last;
    const int nrest = (rest + kMaxF - 1) / kMaxF;
    P.npass = nrest + (last > 0 ? 1 : 0);
    for (int k = 0; k < nrest; ++k) P.F[k] = rest / nrest + (k < rest % nrest ? 1 : 0);
    if (last > 0) P.F[nrest] = last;
  }
  int folded = P.q1;
  Ty prev = P.t1;
  for (int k = 0; k < P.npass; ++k) {
    folded += P.F[k];
    Ty t = P.per_basis ? Ty::F64 : int_type_for(folded, shots);
    if (prev == Ty::F64) t = Ty::F64;
    P.tout[k] = t;
    prev = t;
  }

  // Workspace: ping-pong partial buffers A (counts pass, odd later passes) and B.
  size_t sizeA = 0, sizeB = 0;
  {
    int hh = n - P.q1, ll = P.q1;
    if (P.npass > 0) sizeA = (size_t)(ipow3(hh) << hh) * (size_t)ipow4(ll) * ty_size(P.t1);
    for (int k = 0; k + 1 < P.npass; ++k) {  // outputs of all but the last later pass
      hh -= P.F[k];
      ll += P.F[k];
      size_t sz = (size_t)(ipow3(hh) << hh) * (size_t)ipow4(ll) * ty_size(P.tout[k]);
      if (k % 2 == 0) sizeB = sizeB > sz ? sizeB : sz;
      else sizeA = sizeA > sz ? sizeA : sz;
    }
  }
  const size_t rowpart = (size_t)P.blocks1 * (size_t)ipow3(P.q1) * 4;
  const size_t nbytes = P.per_basis ? (size_t)ipow3(n) * 4 : 0;
  P.J = n < kRhoJ ? n : kRhoJ;
  const size_t tmp = (!(flags & LRE_NO_RHO) && rho_needs_tmp(n)) ? (size_t)ipow4(n) * 16 : 0;

  size_t off = 0;
  P.off_a = off; off += align256(sizeA);
  P.off_b = off; off += align256(sizeB);
  P.off_rowpart = off; off += align256(rowpart);
  P.off_nb = off; off += align256(nbytes);
  P.off_inv = off; off += align256(P.per_basis ? (size_t)ipow3(n) * 8 : 0);
  if (tmp && tmp <= sizeA) P.off_tmp = P.off_a;        // partials are dead by then
  else if (tmp && tmp <= sizeB) P.off_tmp = P.off_b;
  else { P.off_tmp = off; off += align256(tmp); }
  P.total = off;
  return true;
}

// Blocks of `kernel` the device holds at once (compute units x resident blocks per
// unit); a persistent grid of this size has no second wave of blocks.
// lds_bytes: the kernel's static LDS, which bounds the count to 160 KiB per unit.
template <class K>
int64_t resident_blocks(K kernel, int threads, int64_t lds_bytes) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    cus = 256;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu <= 0)
    per_cu = 1;
  const int64_t by_lds = std::max<int64_t>(1, (160 * 1024) / std::max<int64_t>(1, lds_bytes));
  return (int64_t)cus * std::min<int64_t>(per_cu, by_lds);
}

// ---- launch helpers -------------------------------------------------------------

struct Fold1Args {
  const uint16_t* counts;
  int n, chunks;
  int lrow;             // log2 of the row stride of counts (n for a whole instance)
  const uint32_t* nb;   // per-basis totals (MFMA kernel)
  const double* inv;    // their reciprocals (streaming kernel)
  void* out;
  uint32_t* rowpart;
  uint64_t shots;
  int64_t blocks;
  hipStream_t st;
};

// Counts-pass block: one row group per tile row-set, i.e. NRS * LPC threads (3^Q rows
// of 2^Q outcomes); for Q = 7 (81 row-sets of 16 lanes) 432 threads, 27 groups of three
// row-sets each.  (512 threads with uneven step ranges is slower: the groups of a wave
// then flush their row-set sums at different steps and the wave runs both paths.)
template <int Q>
constexpr int fold1_threads() {
  constexpr int t = StreamGeom<Q>::NRS * StreamGeom<Q>::LPC;
  return t > 1024 ? t / 3 : (t < 64 ? 64 : t);
}

// Double-buffered row prefetch with one block per CU (256 registers per lane): faster
// than two blocks per CU without it for 32-bit tiles too (1.04 vs 1.17 ms at n = 12).
template <int Q, typename Acc>
constexpr bool fold1_prefetch() {
  return true;
}

// Waves per SIMD the compiler must leave room for: two blocks per CU when two
// accumulator tiles fit in LDS and the kernel runs without the prefetch, else no
// constraint.
template <int Q, typename Acc>
constexpr int fold1_minwaves() {
  constexpr int waves = (fold1_threads<Q>() + 63) / 64;
  constexpr long lds = (long)StreamGeom<Q>::NACC * (long)sizeof(Acc) + 4L * StreamGeom<Q>::NROWS;
  return (Q == 7 && !fold1_prefetch<Q, Acc>() && 2 * lds <= 160L * 1024) ? (2 * waves + 3) / 4 : 1;
}

template <int Q, typename Acc, bool PB, Out M, bool MAD24>
void launch_fold1(const Fold1Args& a) {
  constexpr int TH = fold1_threads<Q>();
  static_assert(TH <= 1024 && (TH % StreamGeom<Q>::LPC) == 0, "counts-pass block shape");
  hipLaunchKernelGGL((fold_counts_stream_kernel<Q, TH, Acc, PB, M, MAD24, fold1_minwaves<Q, Acc>(),
                                               fold1_prefetch<Q, Acc>()>),
                     dim3((unsigned)a.blocks), dim3(TH), 0,
                     a.st, a.counts, a.n, a.chunks, a.inv, a.out, a.rowpart, a.shots, a.lrow);
}

// The lane butterflies of 32-bit sums use a 24-bit multiply-add when every value they
// see is below 2^23 in magnitude: values are bounded by the counts of the 3^3 rows a
// lane group walks, i.e. by 27 * shots for valid data (rows that exceed `shots` are
// flagged by the row check, so wrong values then never reach the caller as a result).
bool fold1_mad24(uint64_t shots) { return shots > 0 && 27ull * shots < (1ull << 23); }

template <int Q>
bool fold1_q(Ty t, bool pb, Out m, const Fold1Args& a) {
  if (pb) {
    if (m == Out::Partial) launch_fold1<Q, double, true, Out::Partial, false>(a);
    else if (m == Out::CoefPerBasis) launch_fold1<Q, double, true, Out::CoefPerBasis, false>(a);
    else return false;
    return true;
  }
  if (t == Ty::U32) {
    const bool m24 = fold1_mad24(a.shots);
    switch (m) {
      case Out::Partial:
        m24 ? launch_fold1<Q, uint32_t, false, Out::Partial, true>(a)
            : launch_fold1<Q, uint32_t, false, Out::Partial, false>(a);
        return true;
      case Out::CoefUniform:
        m24 ? launch_fold1<Q, uint32_t, false, Out::CoefUniform, true>(a)
            : launch_fold1<Q, uint32_t, false, Out::CoefUniform, false>(a);
        return true;
      case Out::PauliT:
        m24 ? launch_fold1<Q, uint32_t, false, Out::PauliT, true>(a)
            : launch_fold1<Q, uint32_t, false, Out::PauliT, false>(a);
        return true;
      default: return false;
    }
  }
  switch (m) {
    case Out::Partial: launch_fold1<Q, double, false, Out::Partial, false>(a); return true;
    case Out::CoefUniform: launch_fold1<Q, double, false, Out::CoefUniform, false>(a); return true;
    case Out::PauliT: launch_fold1<Q, double, false, Out::PauliT, false>(a); return true;
    default: return false;
  }
}

template <typename Acc, bool PB, Out M>
void launch_fold1_mfma(const Fold1Args& a) {
  constexpr int TH = sizeof(Acc) == 8 ? 512 : 256;
  hipLaunchKernelGGL((fold_counts_mfma_kernel<TH, Acc, PB, M>), dim3((unsigned)a.blocks), dim3(TH), 0,
                     a.st, a.counts, a.n, a.chunks, a.nb, a.out, a.rowpart, a.shots, a.lrow);
}

bool fold1_mfma(Ty t, bool pb, Out m, const Fold1Args& a) {
  if (pb) {
    if (m == Out::Partial) launch_fold1_mfma<double, true, Out::Partial>(a);
    else if (m == Out::CoefPerBasis) launch_fold1_mfma<double, true, Out::CoefPerBasis>(a);
    else return false;
    return true;
  }
  if (t == Ty::U32) {
    switch (m) {
      case Out::Partial: launch_fold1_mfma<uint32_t, false, Out::Partial>(a); return true;
      case Out::CoefUniform: launch_fold1_mfma<uint32_t, false, Out::CoefUniform>(a); return true;
      case Out::PauliT: launch_fold1_mfma<uint32_t, false, Out::PauliT>(a); return true;
      default: return false;
    }
  }
  switch (m) {
    case Out::Partial: launch_fold1_mfma<double, false, Out::Partial>(a); return true;
    case Out::CoefUniform: launch_fold1_mfma<double, false, Out::CoefUniform>(a); return true;
    case Out::PauliT: launch_fold1_mfma<double, false, Out::PauliT>(a); return true;
    default: return false;
  }
}

bool fold1(int q, Ty t, bool pb, Out m, const Fold1Args& a) {
  switch (q) {
    case 1: return fold1_q<1>(t, pb, m, a);
    case 2: return fold1_q<2>(t, pb, m, a);
    case 3: return fold1_q<3>(t, pb, m, a);
    case 4: return fold1_q<4>(t, pb, m, a);
    case 5: return fold1_q<5>(t, pb, m, a);
    case 6: return fold1_q<6>(t, pb, m, a);
    case 7: return fold1_q<7>(t, pb, m, a);
    default: return false;
  }
}

struct FoldKArgs {
  const void* in;
  void* out;
  int n, h, l;
  uint64_t shots;
  int64_t ncols;
  hipStream_t st;
};

template <int F, typename Tin, typename Acc, Out M>
void launch_foldk(const FoldKArgs& a) {
  const int64_t blocks = (a.ncols + 255) / 256;
  hipLaunchKernelGGL((fold_partial_kernel<F, Tin, Acc, M>), dim3((unsigned)blocks), dim3(256), 0, a.st,
                     static_cast<const Tin*>(a.in), a.out, a.n, a.h, a.l, a.shots, a.ncols);
}

template <typename Tin, typename Acc>
void launch_fold4(const FoldKArgs& a) {
  // Persistent blocks: as many as the device holds at once, each walking
  // groups with a stride of the grid.
  const int64_t groups = (ipow3(a.h - 4) << (a.h - 4)) * (((int64_t)1 << (2 * a.l)) / kF4Cols);
  const int64_t cap = resident_blocks(fold_partial4_kernel<Tin, Acc>, 64 * kF4Waves,
                                      (int64_t)256 * kF4Cols * (int64_t)sizeof(Acc));
  const int64_t blocks = groups < cap ? groups : cap;
  hipLaunchKernelGGL((fold_partial4_kernel<Tin, Acc>), dim3((unsigned)blocks), dim3(64 * kF4Waves), 0, a.st,
                     static_cast<const Tin*>(a.in), static_cast<Acc*>(a.out), a.h, a.l);
}

template <int F, typename Tin, typename Acc>
bool foldk_m(Out m, const FoldKArgs& a) {
  if constexpr (F == 4) {         // LDS pass, partials only
    if (m != Out::Partial || a.h < 4 || a.l < 3) return false;
    launch_fold4<Tin, Acc>(a);
    return true;
  } else if constexpr (F > kMaxF) {  // only the final pass writes coefficients
    if (m != Out::Partial) return false;
    launch_foldk<F, Tin, Acc, Out::Partial>(a);
    return true;
  } else {
    switch (m) {
      case Out::Partial: launch_foldk<F, Tin, Acc, Out::Partial>(a); return true;
      case Out::CoefUniform: launch_foldk<F, Tin, Acc, Out::CoefUniform>(a); return true;
      case Out::CoefPerBasis: launch_foldk<F, Tin, Acc, Out::CoefPerBasis>(a); return true;
      case Out::PauliT: launch_foldk<F, Tin, Acc, Out::PauliT>(a); return true;
    }
  }
  return false;
}

template <int F>
bool foldk_f(Ty tin, Ty tacc, Out m, const FoldKArgs& a) {
  if (tin == Ty::U32 && tacc == Ty::U32) return foldk_m<F, uint32_t, uint32_t>(m, a);
  if (tin == Ty::U32 && tacc == Ty::F64) return foldk_m<F, uint32_t, double>(m, a);
  if (tin == Ty::F64 && tacc == Ty::F64) return foldk_m<F, double, double>(m, a);
  return false;
}

bool foldk(int F, Ty tin, Ty tacc, Out m, const FoldKArgs& a) {
  switch (F) {
    case 1: return foldk_f<1>(tin, tacc, m, a);
    case 2: return foldk_f<2>(tin, tacc, m, a);
    case 3: return foldk_f<3>(tin, tacc, m, a);
    case 4: return foldk_f<4>(tin, tacc, m, a);
    default: return false;
  }
}

// Persistent high transform: as many blocks as the LDS lets the device hold.
template <int H, typename OutT>
void launch_rho_high2(const double2* tmp, void* rho, int n, hipStream_t st) {
  using G = RhoHigh2Geom<H>;
  const int64_t items = ((int64_t)1 << H) * G::D * (G::D / G::XB);
  const int64_t blocks =
      std::min<int64_t>(items, resident_blocks(rho_high2_kernel<H, OutT>, 256, 2LL * G::NH * G::SP * 8));
  hipLaunchKernelGGL((rho_high2_kernel<H, OutT>), dim3((unsigned)blocks), dim3(256), 0, st, tmp, rho, n, items);
}

template <int H, int JB, typename OutT>
void launch_rho_real(const double* coef, void* rho, hipStream_t st) {
  using G = RhoRealGeom<H, JB>;
  const int64_t blocks = std::min<int64_t>(
      G::UNITS, resident_blocks(rho_real_tile_kernel<H, JB, OutT>, 512, (int64_t)G::NVP * 8));
  hipLaunchKernelGGL((rho_real_tile_kernel<H, JB, OutT>), dim3((unsigned)blocks), dim3(512), 0, st, coef, rho);
}

template <typename OutT>
void launch_rho(const Plan& P, const double* coef, void* rho, char* ws, hipStream_t st) {
  const int n = P.n;
  if (n <= kRhoJ) {
    switch (n) {
#define LRE_RHO_SMALL(J) \
  case J: hipLaunchKernelGGL((rho_low_kernel<J, true, OutT>), dim3(1), dim3(256), 0, st, coef, rho, n); break;
      LRE_RHO_SMALL(1) LRE_RHO_SMALL(2) LRE_RHO_SMALL(3) LRE_RHO_SMALL(4) LRE_RHO_SMALL(5) LRE_RHO_SMALL(6)
#undef LRE_RHO_SMALL
    }
    return;
  }
  if (n - kRhoJ <= 4) {
    // up to 4 high qubits: units (x_hi, 8 x_lo) from coefficients to mu in LDS
    const dim3 grid((unsigned)((int64_t)8 << (n - kRhoJ)));
    switch (n - kRhoJ) {
      case 1: hipLaunchKernelGGL((rho_tile_kernel<1, OutT>), grid, dim3(512), 0, st, coef, rho); break;
      case 2: hipLaunchKernelGGL((rho_tile_kernel<2, OutT>), grid, dim3(512), 0, st, coef, rho); break;
      case 3: hipLaunchKernelGGL((rho_tile_kernel<3, OutT>), grid, dim3(512), 0, st, coef, rho); break;
      default: hipLaunchKernelGGL((rho_tile_kernel<4, OutT>), grid, dim3(512), 0, st, coef, rho); break;
    }
    return;
  }
  if (n - kRhoJ <= 6) {
    // 5 or 6 high qubits: real-arithmetic units (x_hi, 8 or 4 x_lo), no intermediate
    if (n - kRhoJ == 5) launch_rho_real<5, 3, OutT>(coef, rho, st);
    else launch_rho_real<6, 2, OutT>(coef, rho, st);
    return;
  }
  double2* tmp = reinterpret_cast<double2*>(ws + P.off_tmp);
  const int64_t nblk = ipow4(n - kRhoJ);
  const int64_t low_blocks = std::min<int64_t>(nblk, resident_blocks(rho_low6_kernel, 256, 4096 * 8));
  hipLaunchKernelGGL(rho_low6_kernel, dim3((unsigned)low_blocks), dim3(256), 0, st, coef, tmp, nblk);
  // 7..9 high qubits: two register phases with one LDS transpose
  switch (n - kRhoJ) {
    case 7: launch_rho_high2<7, OutT>(tmp, rho, n, st); break;
    case 8: launch_rho_high2<8, OutT>(tmp, rho, n, st); break;
    default: launch_rho_high2<9, OutT>(tmp, rho, n, st); break;   // n = 15 (streamed estimates)
  }
}


// Per-basis totals N_b of `nbases` rows of 2^lrow counts: the caller's nb_in, else the
// row sums into nb_ws; their reciprocals into inv.  Returns the totals to use.
const uint32_t* prepare_totals(int64_t nbases, int lrow, const uint16_t* counts, const uint32_t* nb_in,
                               uint32_t* nb_ws, double* inv, hipStream_t st) {
  const uint32_t* nb = nb_in;
  if (!nb) {
    hipLaunchKernelGGL(row_totals_kernel, dim3((unsigned)nbases), dim3(256), 0, st, counts, lrow, nb_ws);
    nb = nb_ws;
  }
  hipLaunchKernelGGL(reciprocal_kernel, dim3((unsigned)((nbases + 255) / 256)), dim3(256), 0, st, nb, inv, nbases);
  return nb;
}

// The passes of step (i) over 3^n rows of 2^n counts read with row stride 2^lrow: the
// counts pass (row-sum parts into rowpart) and the later passes, into `final_out` with
// final mode `fm`.  Per-basis mode reads nb (MFMA form) or inv (plain form).
lre_status run_passes(lre_ctx* ctx, const Plan& P, const uint16_t* counts, int lrow, uint64_t shots,
                      const uint32_t* nb, const double* inv, uint32_t* rowpart, void* final_out, Out fm, char* ws,
                      hipStream_t st, bool mfma) {
  const int n = P.n;
  Fold1Args a1{counts, n, P.chunks, lrow, nb, inv, nullptr, rowpart, shots, P.blocks1, st};
  const bool single = P.npass == 0;
  a1.out = single ? final_out : (void*)(ws + P.off_a);
  const bool ok = (mfma && P.q1 == 7) ? fold1_mfma(P.t1, P.per_basis, single ? fm : Out::Partial, a1)
                                       : fold1(P.q1, P.t1, P.per_basis, single ? fm : Out::Partial, a1);
  if (!ok) return LRE_E_UNSUPPORTED;
  if (hipGetLastError() != hipSuccess) return LRE_E_HIP;
  record_stage(ctx, 1, st);

  int h = n - P.q1, l = P.q1;
  Ty tin = P.t1;
  for (int k = 0; k < P.npass; ++k) {
    const bool last = k + 1 == P.npass;
    FoldKArgs ak;
    ak.in = ws + (k % 2 == 0 ? P.off_a : P.off_b);
    ak.out = last ? final_out : (void*)(ws + (k % 2 == 0 ? P.off_b : P.off_a));
    ak.n = n;
    ak.h = h;
    ak.l = l;
    ak.shots = shots;
    ak.ncols = (ipow3(h - P.F[k]) << (h - P.F[k])) * ipow4(l);
    ak.st = st;
    if (!foldk(P.F[k], tin, P.tout[k], last ? fm : Out::Partial, ak)) return LRE_E_UNSUPPORTED;
    if (hipGetLastError() != hipSuccess) return LRE_E_HIP;
    h -= P.F[k];
    l += P.F[k];
    tin = P.tout[k];
  }
  return LRE_OK;
}

// Step (i) into `final_out` (coef or T) with final mode `fm`.
lre_status run_step1(lre_ctx* ctx, const Plan& P, const uint16_t* counts, uint64_t shots,
                     const uint32_t* nb_in, void* final_out, Out fm, char* ws, hipStream_t st,
                     bool mfma) {
  const int n = P.n;
  const int64_t nbases = ipow3(n);
  const uint32_t* nb = nb_in;
  double* inv = nullptr;
  if (P.per_basis) {
    inv = reinterpret_cast<double*>(ws + P.off_inv);
    nb = prepare_totals(nbases, n, counts, nb_in, reinterpret_cast<uint32_t*>(ws + P.off_nb), inv, st);
  }
  uint32_t* rowpart = reinterpret_cast<uint32_t*>(ws + P.off_rowpart);
  const lre_status s = run_passes(ctx, P, counts, n, shots, nb, inv, rowpart, final_out, fm, ws, st, mfma);
  if (s != LRE_OK) return s;

  const int64_t rows = ipow3(P.q1);
  const int64_t runs = ((int64_t)1 << (n - P.q1)) / P.chunks;
  hipLaunchKernelGGL(check_rows_kernel, dim3((unsigned)((nbases + 255) / 256)), dim3(256), 0, st,
                     (const uint32_t*)rowpart, rows, runs, nb, P.per_basis ? (uint64_t)0 : shots, nbases,
                     ctx->flags);
  return hipGetLastError() == hipSuccess ? LRE_OK : LRE_E_HIP;
}

// Steps (i) and (ii) of one instance into caller-given workspace (lre_estimate).
lre_status estimate_impl(lre_ctx* ctx, int n, const uint16_t* counts, uint64_t shots,
                         const uint32_t* n_per_basis, double* coef, void* rho, void* workspace,
                         size_t workspace_bytes, uint32_t flags, void* stream) {
  if (!ctx || !counts || !coef || n < 1 || n > LRE_MAX_QUBITS) return LRE_E_ARG;
  if (flags & ~(LRE_NO_RHO | LRE_RHO_FP32 | LRE_WHT_MFMA)) return LRE_E_ARG;
  if (!aligned(counts, 16) || !aligned(coef, 8)) return LRE_E_ARG;
  const bool want_rho = !(flags & LRE_NO_RHO);
  if (want_rho && (!rho || !aligned(rho, 16))) return LRE_E_ARG;
  Plan P;
  if (!make_plan(n, shots, flags, P)) return LRE_E_ARG;
  if (P.total && (!workspace || !aligned(workspace, 256))) return LRE_E_ARG;
  if (workspace_bytes < P.total) return LRE_E_WORKSPACE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return LRE_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);

  record_stage(ctx, 0, st);
  lre_status s = run_step1(ctx, P, counts, shots, n_per_basis, coef,
                           P.per_basis ? Out::CoefPerBasis : Out::CoefUniform, ws, st,
                           (flags & LRE_WHT_MFMA) != 0);
  if (s != LRE_OK) return s;
  record_stage(ctx, 2, st);
  if (want_rho) {
    if (flags & LRE_RHO_FP32) launch_rho<float>(P, coef, rho, ws, st);
    else launch_rho<double>(P, coef, rho, ws, st);
    if (hipGetLastError() != hipSuccess) return LRE_E_HIP;
  }
  record_stage(ctx, 3, st);
  return LRE_OK;
}

}  // namespace

extern "C" {

const char* lre_status_str(lre_status s) {
  switch (s) {
    case LRE_OK: return "ok";
    case LRE_E_ARG: return "invalid argument";
    case LRE_E_WORKSPACE: return "workspace too small";
    case LRE_E_HIP: return "HIP runtime error";
    case LRE_E_SHOTS: return "a basis row does not sum to its declared total";
    case LRE_E_EMPTY_BASIS: return "a basis has zero counts";
    case LRE_E_UNSUPPORTED: return "unsupported request";
    case LRE_E_TIMEOUT: return "a batched run's bounded wait expired";
    case LRE_E_EIG: return "the eigendecomposition of step (iii) did not converge";
  }
  return "unknown status";
}

lre_status lre_create(lre_ctx** out, int hip_device) {
  if (!out) return LRE_E_ARG;
  *out = nullptr;
  DeviceGuard g(hip_device);
  if (!g.ok) return LRE_E_HIP;
  lre_ctx* c = new (std::nothrow) lre_ctx;
  if (!c) return LRE_E_HIP;
  c->device = hip_device;
  c->flags = nullptr;
  c->n_stage_events = 0;
  for (auto& e : c->stage_events) e = nullptr;
  if (hipMalloc(&c->flags, 64) != hipSuccess) { delete c; return LRE_E_HIP; }
  if (hipMemset(c->flags, 0, 64) != hipSuccess) { (void)hipFree(c->flags); delete c; return LRE_E_HIP; }
  // This device's copy of the static scratch array (device `hip_device` is current).
  void* sp = nullptr;
  const hipError_t se = hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch));
  c->scratch_status = (int)se;
  c->scratch = se == hipSuccess ? static_cast<char*>(sp) : nullptr;
  *out = c;
  return LRE_OK;
}

void lre_destroy(lre_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipFree(ctx->flags);
  lre_detail::destroy_blas(ctx->blas);
  delete ctx;
}

size_t lre_workspace_bytes(int n, uint64_t shots, uint32_t flags) {
  Plan P;
  if (!make_plan(n, shots, flags, P)) return 0;
  return P.total;
}

lre_status lre_estimate(lre_ctx* ctx, int n, const uint16_t* counts, uint64_t shots,
                        const uint32_t* n_per_basis, double* coef, void* rho, void* workspace,
                        size_t workspace_bytes, uint32_t flags, void* stream) {
  return estimate_impl(ctx, n, counts, shots, n_per_basis, coef, rho, workspace, workspace_bytes, flags,
                       stream);
}

lre_status lre_estimate_noalloc(lre_ctx* ctx, int n, const uint16_t* counts, uint64_t shots,
                                const uint32_t* n_per_basis, double* coef, void* rho, uint32_t flags,
                                void* stream) {
  if (!ctx || n < 1 || n > LRE_MAX_QUBITS) return LRE_E_ARG;
  if (lre_workspace_bytes(n, shots, flags) > (size_t)LRE_NOALLOC_SCRATCH_BYTES) return LRE_E_WORKSPACE;
  if (!ctx->scratch) return LRE_E_HIP;
  return estimate_impl(ctx, n, counts, shots, n_per_basis, coef, rho, ctx->scratch,
                       (size_t)LRE_NOALLOC_SCRATCH_BYTES, flags, stream);
}

lre_status lre_set_stage_events(lre_ctx* ctx, void* const* events, int count) {
  if (!ctx || count < 0 || count > 4 || (count > 0 && !events)) return LRE_E_ARG;
  ctx->n_stage_events = events ? count : 0;
  for (int k = 0; k < 4; ++k)
    ctx->stage_events[k] = (events && k < count) ? static_cast<hipEvent_t>(events[k]) : nullptr;
  return LRE_OK;
}

lre_status lre_check(lre_ctx* ctx, void* stream) {
  if (!ctx) return LRE_E_ARG;
  DeviceGuard g(ctx->device);
  if (!g.ok) return LRE_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess) return LRE_E_HIP;
  uint32_t f = 0;
  if (hipMemcpy(&f, ctx->flags, sizeof f, hipMemcpyDeviceToHost) != hipSuccess) return LRE_E_HIP;
  if (f) {
    const uint32_t zero = 0;
    if (hipMemcpy(ctx->flags, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) return LRE_E_HIP;
  }
  if (f & FLAG_WAIT) return LRE_E_TIMEOUT;
  if (f & FLAG_EIG) return LRE_E_EIG;
  if (f & FLAG_ARG) return LRE_E_ARG;
  if (f & FLAG_EMPTY) return LRE_E_EMPTY_BASIS;
  if (f & FLAG_SHOTS) return LRE_E_SHOTS;
  return LRE_OK;
}

lre_status lre_pauli_sums(lre_ctx* ctx, int n, const uint16_t* counts, uint64_t shots, int64_t* T,
                          void* workspace, size_t workspace_bytes, uint32_t flags, void* stream) {
  if (!ctx || !counts || !T || n < 1 || n > LRE_MAX_QUBITS || shots == 0) return LRE_E_ARG;
  if (flags & ~(LRE_NO_RHO | LRE_RHO_FP32 | LRE_WHT_MFMA)) return LRE_E_ARG;
  if (!aligned(counts, 16) || !aligned(T, 8)) return LRE_E_ARG;
  Plan P;
  if (!make_plan(n, shots, flags | LRE_NO_RHO, P)) return LRE_E_ARG;
  if (P.total && (!workspace || !aligned(workspace, 256))) return LRE_E_ARG;
  if (workspace_bytes < P.total) return LRE_E_WORKSPACE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return LRE_E_HIP;
  return run_step1(ctx, P, counts, shots, nullptr, T, Out::PauliT, static_cast<char*>(workspace),
                   static_cast<hipStream_t>(stream), (flags & LRE_WHT_MFMA) != 0);
}

lre_status lre_signed_sums(lre_ctx* ctx, int n, const uint16_t* counts, const int64_t* bases,
                           int64_t num_bases, int32_t* out, uint32_t flags, void* stream) {
  if (!ctx || !counts || !bases || !out || n < 1 || n > LRE_MAX_QUBITS || num_bases < 0)
    return LRE_E_ARG;
  if (flags & ~(LRE_WHT_MFMA)) return LRE_E_ARG;
  if ((flags & LRE_WHT_MFMA) && n < 6) return LRE_E_UNSUPPORTED;
  if (!aligned(counts, 16) || !aligned(out, 4) || !aligned(bases, 8)) return LRE_E_ARG;
  if (num_bases == 0) return LRE_OK;
  if (num_bases > INT32_MAX) return LRE_E_ARG;
  DeviceGuard g(ctx->device);
  if (!g.ok) return LRE_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t lds = (size_t)4 << n;
  if (flags & LRE_WHT_MFMA) {
    hipLaunchKernelGGL(signed_sums_mfma_kernel, dim3((unsigned)num_bases), dim3(256), lds, st, counts, n, bases, out,
                       ctx->flags);
    return hipGetLastError() == hipSuccess ? LRE_OK : LRE_E_HIP;
  }
  const int q = n < kMaxQ1 ? n : kMaxQ1;
  switch (q) {
#define LRE_SS(Q)                                                                                  \
  case Q:                                                                                          \
    hipLaunchKernelGGL(signed_sums_kernel<Q>, dim3((unsigned)num_bases), dim3(256), lds, st, counts, n, \
                       bases, out, ctx->flags);                                                    \
    break;
    LRE_SS(1) LRE_SS(2) LRE_SS(3) LRE_SS(4) LRE_SS(5) LRE_SS(6) LRE_SS(7)
#undef LRE_SS
  }
  return hipGetLastError() == hipSuccess ? LRE_OK : LRE_E_HIP;
}


// ---------------------------------------------------------------------------------
// Streamed estimation (lre_stream_*): slabs of 3^(n-h) consecutive bases, each cut
// into 2^h outcome segments run as (n-h)-qubit instances, the top h qubits folded into
// the caller's coefficient array, which accumulates until lre_stream_finish.

}  // extern "C"

struct lre_stream {
  lre_ctx* ctx = nullptr;
  int n = 0, h = 0, np = 0;
  uint64_t shots = 0;
  uint32_t flags = 0;
  Plan P;                     // plan of one (n-h)-qubit segment (no rho), final sums raw
  Ty tV = Ty::F64;            // type of the segments' final sums
  int64_t slabs = 0;          // 3^h
  std::vector<uint8_t> pushed;
  int64_t npushed = 0;
  double* coef = nullptr;     // accumulator / output, set by lre_stream_begin
  size_t off_seg = 0, off_V = 0, off_rowpart = 0, off_stage = 0, off_tmp = 0, total = 0;
  size_t seg_rowpart = 0;     // bytes of one segment's row-sum parts
  size_t stage_bytes = 0;
  hipEvent_t copied = nullptr;
};

namespace {

lre_status stream_ws_check(const lre_stream* S, void* ws, size_t ws_bytes) {
  if (!ws || !aligned(ws, 256)) return LRE_E_ARG;
  if (ws_bytes < S->total) return LRE_E_WORKSPACE;
  return LRE_OK;
}

template <int H>
void launch_top_fold(const lre_stream* S, const void* V, uint32_t atop, hipStream_t st) {
  const int64_t ncols = ipow4(S->np);
  const dim3 grid((unsigned)((ncols + 255) / 256));
  if (S->tV == Ty::U32)
    hipLaunchKernelGGL((stream_top_fold_kernel<H, uint32_t>), grid, dim3(256), 0, st, (const uint32_t*)V, S->coef,
                       ncols, atop);
  else
    hipLaunchKernelGGL((stream_top_fold_kernel<H, double>), grid, dim3(256), 0, st, (const double*)V, S->coef,
                       ncols, atop);
}

// One slab already in device memory: totals, the 2^h segments, the row check, the fold
// of the top qubits into the accumulator.
lre_status stream_slab(lre_stream* S, int64_t slab, const uint16_t* counts, const uint32_t* nb_in, char* ws,
                       hipStream_t st) {
  const Plan& P = S->P;
  const int np = S->np, n = S->n, h = S->h;
  const int64_t nbases = ipow3(np);
  char* seg_ws = ws + S->off_seg;
  const uint32_t* nb = nb_in;
  double* inv = nullptr;
  if (P.per_basis) {
    inv = reinterpret_cast<double*>(seg_ws + P.off_inv);
    nb = prepare_totals(nbases, n, counts, nb_in, reinterpret_cast<uint32_t*>(seg_ws + P.off_nb), inv, st);
  }
  const size_t vbytes = (size_t)ipow4(np) * ty_size(S->tV);
  for (int sg = 0; sg < (1 << h); ++sg) {
    uint32_t* rowpart = reinterpret_cast<uint32_t*>(ws + S->off_rowpart + (size_t)sg * S->seg_rowpart);
    void* V = ws + S->off_V + (size_t)sg * vbytes;
    const lre_status s = run_passes(S->ctx, P, counts + ((int64_t)sg << np), n, S->shots, nb, inv, rowpart, V,
                                    Out::Partial, seg_ws, st, (S->flags & LRE_WHT_MFMA) != 0);
    if (s != LRE_OK) return s;
  }
  const int64_t rows = ipow3(P.q1);
  const int64_t runs = ((int64_t)1 << (np - P.q1)) / P.chunks;
  hipLaunchKernelGGL(check_rows_seg_kernel, dim3((unsigned)((nbases + 255) / 256)), dim3(256), 0, st,
                     (const uint32_t*)(ws + S->off_rowpart), (int64_t)(S->seg_rowpart / 4), 1 << h, rows, runs, nb,
                     P.per_basis ? (uint64_t)0 : S->shots, nbases, S->ctx->flags);
  // Letters of the top qubits: digit p of the slab index (base 3) is qubit h - p.
  uint32_t atop = 0;
  int64_t t = slab;
  for (int p = 0; p < h; ++p) {
    atop |= (uint32_t)(t % 3 + 1) << (2 * p);
    t /= 3;
  }
  const void* V = ws + S->off_V;
  switch (h) {
    case 1: launch_top_fold<1>(S, V, atop, st); break;
    case 2: launch_top_fold<2>(S, V, atop, st); break;
    case 3: launch_top_fold<3>(S, V, atop, st); break;
    case 4: launch_top_fold<4>(S, V, atop, st); break;
    case 5: launch_top_fold<5>(S, V, atop, st); break;
    default: launch_top_fold<6>(S, V, atop, st); break;
  }
  return hipGetLastError() == hipSuccess ? LRE_OK : LRE_E_HIP;
}

lre_status stream_take_slab(lre_stream* S, int64_t slab) {
  if (!S->coef) return LRE_E_ARG;                       // lre_stream_begin first
  if (slab < 0 || slab >= S->slabs || S->pushed[(size_t)slab]) return LRE_E_ARG;
  S->pushed[(size_t)slab] = 1;
  ++S->npushed;
  return LRE_OK;
}

}  // namespace

extern "C" {

lre_status lre_stream_create(lre_ctx* ctx, int n, int h, uint64_t shots, uint32_t flags, lre_stream** out) {
  if (!out) return LRE_E_ARG;
  *out = nullptr;
  if (!ctx || n > LRE_STREAM_MAX_QUBITS || h < 1 || h > 6 || n - h < 8 || n - h > LRE_MAX_QUBITS)
    return LRE_E_ARG;
  if (flags & ~(LRE_NO_RHO | LRE_RHO_FP32 | LRE_WHT_MFMA | LRE_STREAM_HOST)) return LRE_E_ARG;
  lre_stream* S = new (std::nothrow) lre_stream;
  if (!S) return LRE_E_HIP;
  S->ctx = ctx;
  S->n = n;
  S->h = h;
  S->np = n - h;
  S->shots = shots;
  S->flags = flags;
  if (!make_plan(S->np, shots, (flags & LRE_WHT_MFMA) | LRE_NO_RHO, S->P)) {
    delete S;
    return LRE_E_ARG;
  }
  S->tV = S->P.npass ? S->P.tout[S->P.npass - 1] : S->P.t1;
  S->slabs = ipow3(h);
  S->pushed.assign((size_t)S->slabs, 0);
  const size_t segs = (size_t)1 << h;
  S->seg_rowpart = align256((size_t)S->P.blocks1 * (size_t)ipow3(S->P.q1) * 4);
  size_t off = 0;
  S->off_seg = off; off += align256(S->P.total);
  S->off_V = off; off += align256(segs * (size_t)ipow4(S->np) * ty_size(S->tV));
  S->off_rowpart = off; off += segs * S->seg_rowpart;
  S->stage_bytes = (size_t)ipow3(S->np) << n;
  S->stage_bytes *= 2;
  if (flags & LRE_STREAM_HOST) {
    S->off_stage = off;
    off += align256(S->stage_bytes);
    off += align256(S->P.per_basis ? (size_t)ipow3(S->np) * 4 : 0);   // staged N_b
  }
  // step (ii)'s intermediate reuses the (then dead) segment buffers
  const size_t tmp = (flags & LRE_NO_RHO) ? 0 : (size_t)ipow4(n) * 16;
  S->off_tmp = 0;
  S->total = off > tmp ? off : tmp;
  DeviceGuard g(ctx->device);
  if (!g.ok || hipEventCreateWithFlags(&S->copied, hipEventDisableTiming) != hipSuccess) {
    delete S;
    return LRE_E_HIP;
  }
  *out = S;
  return LRE_OK;
}

size_t lre_stream_workspace_bytes(const lre_stream* S) { return S ? S->total : 0; }

lre_status lre_stream_begin(lre_stream* S, double* coef, void* workspace, size_t workspace_bytes, void* stream) {
  if (!S || !coef || !aligned(coef, 8)) return LRE_E_ARG;
  const lre_status c = stream_ws_check(S, workspace, workspace_bytes);
  if (c != LRE_OK) return c;
  DeviceGuard g(S->ctx->device);
  if (!g.ok) return LRE_E_HIP;
  S->coef = coef;
  std::fill(S->pushed.begin(), S->pushed.end(), 0);
  S->npushed = 0;
  // the accumulator starts at zero (a fill kernel: capturable, no memset node)
  const int64_t words = ipow4(S->n) * 2;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((words + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), reinterpret_cast<uint32_t*>(coef), words, 0u);
  return hipGetLastError() == hipSuccess ? LRE_OK : LRE_E_HIP;
}

lre_status lre_stream_push(lre_stream* S, int64_t slab, const uint16_t* counts, const uint32_t* n_per_basis,
                           void* workspace, size_t workspace_bytes, void* stream) {
  if (!S || !counts || !aligned(counts, 16)) return LRE_E_ARG;
  if (n_per_basis && !aligned(n_per_basis, 4)) return LRE_E_ARG;
  lre_status c = stream_ws_check(S, workspace, workspace_bytes);
  if (c != LRE_OK) return c;
  if ((c = stream_take_slab(S, slab)) != LRE_OK) return c;
  DeviceGuard g(S->ctx->device);
  if (!g.ok) return LRE_E_HIP;
  return stream_slab(S, slab, counts, S->P.per_basis ? n_per_basis : nullptr, static_cast<char*>(workspace),
                     static_cast<hipStream_t>(stream));
}

lre_status lre_stream_push_host(lre_stream* S, int64_t slab, const uint16_t* counts, const uint32_t* n_per_basis,
                                void* workspace, size_t workspace_bytes, void* stream) {
  if (!S || !counts) return LRE_E_ARG;
  if (!(S->flags & LRE_STREAM_HOST)) return LRE_E_ARG;
  lre_status c = stream_ws_check(S, workspace, workspace_bytes);
  if (c != LRE_OK) return c;
  if (slab < 0 || slab >= S->slabs || S->pushed[(size_t)slab] || !S->coef) return LRE_E_ARG;
  DeviceGuard g(S->ctx->device);
  if (!g.ok) return LRE_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  uint16_t* stage = reinterpret_cast<uint16_t*>(ws + S->off_stage);
  uint32_t* nb_stage = nullptr;
  // The staging buffer is reused by every slab: the copy is ordered after the previous
  // slab's kernels on the same stream.
  if (hipMemcpyAsync(stage, counts, S->stage_bytes, hipMemcpyHostToDevice, st) != hipSuccess) return LRE_E_HIP;
  if (S->P.per_basis && n_per_basis) {
    nb_stage = reinterpret_cast<uint32_t*>(ws + S->off_stage + align256(S->stage_bytes));
    if (hipMemcpyAsync(nb_stage, n_per_basis, (size_t)ipow3(S->np) * 4, hipMemcpyHostToDevice, st) != hipSuccess)
      return LRE_E_HIP;
  }
  if (hipEventRecord(S->copied, st) != hipSuccess) return LRE_E_HIP;
  if ((c = stream_take_slab(S, slab)) != LRE_OK) return c;
  c = stream_slab(S, slab, stage, nb_stage, ws, st);
  if (c != LRE_OK) return c;
  // the caller may reuse its host buffers once the copies are done (the slab's kernels
  // keep running)
  return hipEventSynchronize(S->copied) == hipSuccess ? LRE_OK : LRE_E_HIP;
}

lre_status lre_stream_finish(lre_stream* S, void* rho, void* workspace, size_t workspace_bytes, void* stream) {
  if (!S || !S->coef) return LRE_E_ARG;
  if (S->npushed != S->slabs) return LRE_E_ARG;
  const bool want_rho = !(S->flags & LRE_NO_RHO);
  if (want_rho && (!rho || !aligned(rho, 16))) return LRE_E_ARG;
  const lre_status c = stream_ws_check(S, workspace, workspace_bytes);
  if (c != LRE_OK) return c;
  DeviceGuard g(S->ctx->device);
  if (!g.ok) return LRE_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t count = ipow4(S->n);
  hipLaunchKernelGGL(stream_finish_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, S->coef, S->n,
                     S->P.per_basis ? (uint64_t)0 : S->shots, count);
  if (hipGetLastError() != hipSuccess) return LRE_E_HIP;
  if (want_rho) {
    Plan R;
    R.n = S->n;
    R.off_tmp = S->off_tmp;
    if (S->flags & LRE_RHO_FP32) launch_rho<float>(R, S->coef, rho, static_cast<char*>(workspace), st);
    else launch_rho<double>(R, S->coef, rho, static_cast<char*>(workspace), st);
    if (hipGetLastError() != hipSuccess) return LRE_E_HIP;
  }
  S->coef = nullptr;
  return LRE_OK;
}

void lre_stream_destroy(lre_stream* S) {
  if (!S) return;
  {
    DeviceGuard g(S->ctx->device);
    if (S->copied) (void)hipEventDestroy(S->copied);
  }
  delete S;
}


// ---------------------------------------------------------------------------------
// Reduced measurement set (Sec. VI): 4^n product operators of one informationally
// complete 4-operator set per qubit.

size_t lre_povm_workspace_bytes(int n, uint32_t flags) {
  if (n < 1 || n > LRE_MAX_QUBITS) return 0;
  const size_t head = 256;   // M (16 binary64) and the 64-bit total N
  const size_t tmp = (!(flags & LRE_NO_RHO) && rho_needs_tmp(n)) ? (size_t)ipow4(n) * 16 : 0;
  return head + align256(tmp);
}

lre_status lre_povm_estimate(lre_ctx* ctx, int n, const uint16_t* counts, const double* G, double* coef, void* rho,
                             void* workspace, size_t workspace_bytes, uint32_t flags, void* stream) {
  if (!ctx || !counts || !G || !coef || n < 1 || n > LRE_MAX_QUBITS) return LRE_E_ARG;
  if (flags & ~(LRE_NO_RHO | LRE_RHO_FP32)) return LRE_E_ARG;
  if (!aligned(counts, 16) || !aligned(G, 8) || !aligned(coef, 8)) return LRE_E_ARG;
  const bool want_rho = !(flags & LRE_NO_RHO);
  if (want_rho && (!rho || !aligned(rho, 16))) return LRE_E_ARG;
  const size_t need = lre_povm_workspace_bytes(n, flags);
  if (!workspace || !aligned(workspace, 256)) return LRE_E_ARG;
  if (workspace_bytes < need) return LRE_E_WORKSPACE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return LRE_E_HIP;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  double* M = reinterpret_cast<double*>(ws);
  unsigned long long* total = reinterpret_cast<unsigned long long*>(ws + 128);
  const int64_t count = ipow4(n);

  record_stage(ctx, 0, st);
  hipLaunchKernelGGL(povm_setup_kernel, dim3(1), dim3(64), 0, st, G, M, total, ctx->flags);
  record_stage(ctx, 1, st);

  // passes: the lowest min(n, 6) digits in one LDS tile (which also sums the counts into
  // N), then 4 digits at a time in LDS, then the remaining 1..3 in registers; the last
  // pass divides by N
  const int J = n < 6 ? n : 6;
  const int64_t tiles = count >> (2 * J);
  const bool only = J == n;
  switch (J) {
#define LRE_POVM_LOW(JJ)                                                                                   \
  case JJ:                                                                                                 \
    if (only)                                                                                              \
      hipLaunchKernelGGL((povm_low_kernel<JJ, true>), dim3((unsigned)tiles), dim3(256), 0, st, counts, coef, \
                         (const double*)M, total, ctx->flags);                                              \
    else                                                                                                   \
      hipLaunchKernelGGL((povm_low_kernel<JJ, false>), dim3((unsigned)tiles), dim3(256), 0, st, counts, coef, \
                         (const double*)M, total, ctx->flags);                                              \
    break;
    LRE_POVM_LOW(1) LRE_POVM_LOW(2) LRE_POVM_LOW(3) LRE_POVM_LOW(4) LRE_POVM_LOW(5) LRE_POVM_LOW(6)
#undef LRE_POVM_LOW
  }
  if (!only)
    hipLaunchKernelGGL(povm_check_kernel, dim3(1), dim3(64), 0, st, (const unsigned long long*)total, ctx->flags);
  int lo = J;
  while (n - lo >= 4) {
    const bool last = n - lo == 4;
    const int64_t blocks = (count >> 8) / kPovmCols;
    if (last)
      hipLaunchKernelGGL((povm_high4_kernel<true>), dim3((unsigned)blocks), dim3(kPovmHighThreads), 0, st, coef, n,
                         lo, (const double*)M, (const unsigned long long*)total);
    else
      hipLaunchKernelGGL((povm_high4_kernel<false>), dim3((unsigned)blocks), dim3(kPovmHighThreads), 0, st, coef, n,
                         lo, (const double*)M, (const unsigned long long*)total);
    lo += 4;
  }
  if (n > lo) {
    const int F = n - lo;
    const int64_t cols = count >> (2 * F);
    const dim3 grid((unsigned)((cols + 255) / 256));
    switch (F) {
      case 1: hipLaunchKernelGGL((povm_reg_kernel<1, true>), grid, dim3(256), 0, st, coef, n, lo, (const double*)M, (const unsigned long long*)total); break;
      case 2: hipLaunchKernelGGL((povm_reg_kernel<2, true>), grid, dim3(256), 0, st, coef, n, lo, (const double*)M, (const unsigned long long*)total); break;
      default: hipLaunchKernelGGL((povm_reg_kernel<3, true>), grid, dim3(256), 0, st, coef, n, lo, (const double*)M, (const unsigned long long*)total); break;
    }
  }
  if (hipGetLastError() != hipSuccess) return LRE_E_HIP;
  record_stage(ctx, 2, st);
  if (want_rho) {
    Plan R;
    R.n = n;
    R.off_tmp = 256;
    if (flags & LRE_RHO_FP32) launch_rho<float>(R, coef, rho, ws, st);
    else launch_rho<double>(R, coef, rho, ws, st);
    if (hipGetLastError() != hipSuccess) return LRE_E_HIP;
  }
  record_stage(ctx, 3, st);
  return LRE_OK;
}

}  // extern "C"
