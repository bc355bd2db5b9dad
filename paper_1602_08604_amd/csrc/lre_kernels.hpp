// lre_kernels.hpp -- gfx950 kernels for LRE steps (i) and (ii).
//
// Step (i) (Sec. II eq. 3 with the Pauli structure of Sec. III) is the tensor map
//   T = ((x)_k B) c,  B = 4x6 integer matrix on one qubit's (basis letter, outcome bit),
// whose rows are the one-qubit Gamma vectors (times sqrt 2) of Sec. III:
//   a = I : +1 for every (letter, outcome)            (the Gamma_0 entries)
//   a = X : +1 / -1 on (X, +) / (X, -), 0 elsewhere    (likewise Y, Z)
// B factors as (sum-or-select over the 3 letters) . (2-point Hadamard on the outcome
// bit), so a qubit is "folded" by a Walsh-Hadamard butterfly on its outcome bit
// followed by: I <- sum over letters of the even part, X/Y/Z <- the odd part of the
// matching letter.  Folding a group of qubits turns 6 values per qubit into 4.
// (X^T X)^{-1} = (x)_k diag{1/3,1,1,1} is applied once at the end as a division by
// 3^{n-w(i)} (w = number of non-identity letters).
//
// Tensor layout between passes (row-major, mixed radix):
//   [b_hi : 3^h][s_hi : 2^h][a_lo : 4^l]
// h qubits still raw (basis letter digits, outcome bits), l qubits folded into
// Pauli letters.  Qubit positions count from the least significant (position p has
// weight 3^p in b, 2^p in s, 4^p in the Pauli index), so the lowest qubits fold first.
//
// Pass 1 (counts_block / fold_counts_stream_kernel) streams the uint16 counts once and
// folds the lowest Q <= 7 qubits: a tile is 3^Q rows x 2^Q consecutive outcomes; a lane
// owns 8 outcomes of a row, a group of 16 lanes walks 27 rows, folds the 3 register
// qubits with an accumulator cascade, applies the lane butterflies to the values that
// leave the cascade and adds them into a 4^Q LDS accumulator.  Later passes
// (fold_partial_col / fold_partial_kernel) fold up to 3 more qubits per pass, one
// thread per column of the fastest-varying a_lo index, entirely in registers, or 4
// (fold_partial4_kernel) with the letter codes of 64 columns accumulated in LDS.
//
// Step (ii) (Sec. II eq. 4): with x = r XOR c, the entry mu[r][r^x] is a Walsh-Hadamard
// transform over z in {0,1}^n of e_{a(x,z)} (-i)^{|x&z|}, where per qubit the pair
// (x_k, z_k) = (0,0),(1,0),(1,1),(0,1) is the letter I, X, Y, Z (the paper's grouping of
// the Omega_i by nonzero pattern, Sec. IV).  n <= 6: rho_low_kernel does all of it in
// LDS.  7 <= n <= 10: rho_tile_kernel, units of one high pattern and 8 low patterns
// from coefficients to mu in LDS (a real low transform, the complex one rebuilt from
// pairs of its outputs, the high transform in registers).  n = 11, 12:
// rho_real_tile_kernel, the whole n-qubit transform real (the sign (-1)^{floor(|x&z|/2)}
// applied on input) and the complex entry rebuilt from the outputs at r and r^x, units
// of one high pattern and 8 or 4 low patterns in LDS.  n > 12: rho_low6_kernel
// transforms the low 6 qubits of each 4^6 coefficient block (registers + lane quads)
// into a complex intermediate, then rho_high2_kernel (5 to 9 high qubits, two register
// phases and one LDS transpose) the remaining high qubits, writing the row-major
// matrix.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lre {

__host__ __device__ constexpr int64_t ipow3(int k) { return k <= 0 ? 1 : 3 * ipow3(k - 1); }
__host__ __device__ constexpr int64_t ipow4(int k) { return k <= 0 ? 1 : 4 * ipow4(k - 1); }
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

enum : uint32_t { FLAG_SHOTS = 1u, FLAG_EMPTY = 2u, FLAG_ARG = 4u, FLAG_WAIT = 8u, FLAG_EIG = 16u };

// What the final pass writes.
enum class Out : int { Partial = 0, CoefUniform = 1, CoefPerBasis = 2, PauliT = 3 };

// Number of non-identity letters of a Pauli index (base-4 digits).
__device__ __forceinline__ int pauli_weight(uint64_t a) {
  return __popcll((a | (a >> 1)) & 0x5555555555555555ull);
}

// 3^k as an exact binary64 (k <= 33).
__device__ __forceinline__ double pow3d(int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= 3.0;
  return r;
}

// Compile-time helpers for the register fold of RD basis digits.
// Letter digit of position p in a small Pauli index ar, and base-3 digit of beta.
__host__ __device__ constexpr int adig(int ar, int p) { return (ar >> (2 * p)) & 3; }
__host__ __device__ constexpr int bdig(int beta, int p) { return p == 0 ? beta % 3 : bdig(beta / 3, p - 1); }
// Walsh index bits selected by ar: bit p set iff letter p is not the identity.
__host__ __device__ constexpr int mlo_of(int ar, int rd) {
  return rd == 0 ? 0 : (mlo_of(ar, rd - 1) | ((adig(ar, rd - 1) != 0) << (rd - 1)));
}
// Does basis row beta contribute to Pauli letters ar on the rd lowest positions?
__host__ __device__ constexpr bool compat(int beta, int ar, int rd) {
  return rd == 0 ? true
                 : (compat(beta, ar, rd - 1) &&
                    (adig(ar, rd - 1) == 0 || adig(ar, rd - 1) == bdig(beta, rd - 1) + 1));
}

// Value of the Pauli index restricted to the positions of a folded block, for basis
// digits beta (base 3) and Walsh index m (base 2) of F positions.
__host__ __device__ constexpr int fold_index(int beta, int m, int f) {
  return f == 0 ? 0
                : (fold_index(beta, m, f - 1) |
                   ((((m >> (f - 1)) & 1) ? (bdig(beta, f - 1) + 1) : 0) << (2 * (f - 1))));
}

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int B, int E>
struct StaticFor {
  template <class Fn>
  __device__ __forceinline__ static void run(Fn&& f) {
    if constexpr (B < E) {
      f(std::integral_constant<int, B>{});
      StaticFor<B + 1, E>::run(f);
    }
  }
};

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also fences global
// memory, which makes every wave wait for all of its outstanding loads (prefetches
// included) at the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------------
// Walsh-Hadamard butterflies.  Natural order: after the transform element m holds
// sum_s x_s (-1)^{popcount(s & m)}.

template <int NB, typename T>
__device__ __forceinline__ void wht_regs(T* x) {
#pragma unroll
  for (int bit = 0; bit < NB; ++bit) {
#pragma unroll
    for (int v = 0; v < (1 << NB); ++v) {
      if (v & (1 << bit)) continue;
      T a = x[v], b = x[v | (1 << bit)];
      x[v] = a + b;
      x[v | (1 << bit)] = a - b;
    }
  }
}

// Butterflies across the NL low bits of the lane index (groups of 2^NL <= 16
// consecutive lanes), on the VALU through DPP (no LDS traffic).  gfx9 DPP offers
// quad_perm (partners lane^1, lane^2 within a quad), row_half_mirror (lane^7 within
// 8) and row_mirror (lane^15 within 16).  A stage along direction v pairs lane i with
// i^v; the member with odd parity of (i & U) keeps partner - x, the other x + partner.
// With the directions and masks U below the stages compose to the exact Walsh-Hadamard
// transform over the lane bits with the output index relabelled by a linear map
// sigma (checked exhaustively on the host): lane l ends up holding Walsh index
// lane_walsh<NL>(l) for its lane bits.
//   NL = 1, 2 : lane^1 (U = 1), lane^2 (U = 2)                  sigma = identity
//   NL = 3    : lane^7 (U = 4), lane^1 (U = 5), lane^2 (U = 6)   sigma(1,2,4) = 5,6,7
//   NL = 4    : lane^15 (U = 8), lane^7 (U = 12), lane^1 (U = 5), lane^2 (U = 6)
//                                                               sigma(1,2,4,8) = 5,6,15,4
template <int NL>
__host__ __device__ constexpr int lane_walsh(int l) {
  if constexpr (NL <= 2) {
    return l;
  } else if constexpr (NL == 3) {
    return ((l & 1) ? 5 : 0) ^ ((l & 2) ? 6 : 0) ^ ((l & 4) ? 7 : 0);
  } else {
    return ((l & 1) ? 5 : 0) ^ ((l & 2) ? 6 : 0) ^ ((l & 4) ? 15 : 0) ^ ((l & 8) ? 4 : 0);
  }
}

constexpr int kDppQuadXor1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int kDppQuadXor2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppMirror = 0x140;     // row_mirror

// Values here are partial Walsh sums of at most 2^7 uint16 counts, |x| < 2^23, so the
// +-1 weighting is a 24-bit signed multiply-add (v_mad_i32_i24) behind the DPP move.
template <int CTRL, int V>
__device__ __forceinline__ void lane_stage(int32_t* x, int lam, int umask) {
  int32_t sgn = (__popc((unsigned)(lam & umask)) & 1) ? -1 : 1;  // partner - x for the odd member
  // Hide the +-1 range from the optimiser, which would otherwise expand the multiply
  // into select/negate sequences (3-4 VALU ops instead of one v_mad_i32_i24).
  asm volatile("" : "+v"(sgn));
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const int32_t p = __builtin_amdgcn_mov_dpp(x[v], CTRL, 0xF, 0xF, true);
    x[v] = __mul24(x[v], sgn) + p;
  }
}

template <int NL, int V>
__device__ __forceinline__ void wht_lanes(int32_t* x, int lam) {
  if constexpr (NL == 1) {
    lane_stage<kDppQuadXor1, V>(x, lam, 1);
  } else if constexpr (NL == 2) {
    lane_stage<kDppQuadXor1, V>(x, lam, 1);
    lane_stage<kDppQuadXor2, V>(x, lam, 2);
  } else if constexpr (NL == 3) {
    lane_stage<kDppHalfMirror, V>(x, lam, 4);
    lane_stage<kDppQuadXor1, V>(x, lam, 5);
    lane_stage<kDppQuadXor2, V>(x, lam, 6);
  } else if constexpr (NL == 4) {
    lane_stage<kDppMirror, V>(x, lam, 8);
    lane_stage<kDppHalfMirror, V>(x, lam, 12);
    lane_stage<kDppQuadXor1, V>(x, lam, 5);
    lane_stage<kDppQuadXor2, V>(x, lam, 6);
  }
}

// ---------------------------------------------------------------------------------
// Row tiles of the counts: 2^Q consecutive outcomes of a row, V per lane.

template <int Q>
struct Fold1Geom {
  static constexpr int V = Q >= 3 ? 8 : (1 << Q);  // outcomes per lane
  static constexpr int LB = ilog2c(V);              // Walsh bits held in registers
  static constexpr int LPC = (1 << Q) / V;          // lanes per tile row
  static constexpr int LL = Q - LB;                 // Walsh bits across lanes
};

template <int V>
__device__ __forceinline__ void load_counts(const uint16_t* __restrict__ p, int32_t* x) {
  if constexpr (V == 8) {
    uint4 w = *reinterpret_cast<const uint4*>(p);
    uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) { x[2 * k] = (int32_t)(u[k] & 0xffffu); x[2 * k + 1] = (int32_t)(u[k] >> 16); }
  } else if constexpr (V == 4) {
    uint2 w = *reinterpret_cast<const uint2*>(p);
    x[0] = (int32_t)(w.x & 0xffffu); x[1] = (int32_t)(w.x >> 16);
    x[2] = (int32_t)(w.y & 0xffffu); x[3] = (int32_t)(w.y >> 16);
  } else {
    uint32_t w = *reinterpret_cast<const uint32_t*>(p);
    x[0] = (int32_t)(w & 0xffffu); x[1] = (int32_t)(w >> 16);
  }
}

// Counts are read once per step: the 16-byte loads carry the nontemporal hint so the
// stream does not evict lines other blocks still need (n = 12 counts pass 1.04 -> 0.87 ms).
template <int V>
__device__ __forceinline__ void load_raw(const uint16_t* __restrict__ p, uint32_t* w) {
  if constexpr (V == 8) {
    typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
    const u32x4_t u = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p));
    w[0] = u.x; w[1] = u.y; w[2] = u.z; w[3] = u.w;
  } else if constexpr (V == 4) {
    const uint2 u = *reinterpret_cast<const uint2*>(p);
    w[0] = u.x; w[1] = u.y;
  } else {
    w[0] = *reinterpret_cast<const uint32_t*>(p);
  }
}

template <int V>
__device__ __forceinline__ void unpack_raw(const uint32_t* w, int32_t* x) {
#pragma unroll
  for (int k = 0; k < V / 2; ++k) { x[2 * k] = (int32_t)(w[k] & 0xffffu); x[2 * k + 1] = (int32_t)(w[k] >> 16); }
}

// Accumulator conversion of an exact chunk sum.
template <typename Acc>
__device__ __forceinline__ Acc to_acc(int32_t s) {
  if constexpr (sizeof(Acc) == 4) return (Acc)(uint32_t)s;  // wrap-around integer
  else return (Acc)s;
}

template <typename Acc>
__device__ __forceinline__ double acc_to_double(Acc v) {
  if constexpr (sizeof(Acc) == 4) return (double)(int32_t)(uint32_t)v;
  else return (double)v;
}

template <typename Acc>
__device__ __forceinline__ int64_t acc_to_i64(Acc v) {
  if constexpr (sizeof(Acc) == 4) return (int64_t)(int32_t)(uint32_t)v;
  else return (int64_t)v;
}

// ---------------------------------------------------------------------------------
// Pass 1 (counts pass): counts -> partials (or the final coefficients when Q == n).
// A block tile is 3^Q rows x 2^Q consecutive outcomes (V = 8 outcomes per lane, LPC
// lanes per tile row).  The per-qubit maps act on different qubits and commute, so
// they are applied in the order that keeps most of the work in registers:
//   1. each lane walks the 3^LB rows that differ in the basis digits of the LB qubits
//      whose outcome bits it holds in registers, doing the in-register butterflies and
//      folding those LB qubits completely with a mixed-radix cascade of accumulators
//      (level k holds the identity-letter sums of qubit k);
//   2. only the 4^LB values that leave the cascade ("emissions", one per letter
//      combination of those qubits) get the lane butterflies (DPP) of the remaining
//      LL = Q - LB outcome bits and are added into the LDS accumulator, whose atomics
//      fold the last LL qubits over the row-sets.
// Per 27 rows x 8 outcomes a lane issues 64 emissions: 0.30 LDS atomics per count and
// the DPP work runs on 30% of the values.

// One DPP butterfly stage on a 32-bit integer value: lower member x + partner, upper
// partner - x.  MAD24: |x| < 2^23 is guaranteed by the caller (v_mad_i32_i24);
// otherwise an exact negate-and-add.
template <int CTRL, bool MAD24>
__device__ __forceinline__ void lane_bfly(int32_t& x, int32_t sgn) {
  const int32_t p = __builtin_amdgcn_mov_dpp(x, CTRL, 0xF, 0xF, true);
  if constexpr (MAD24) {
    x = __mul24(x, sgn) + p;
  } else {
    const int32_t neg = sgn >> 31;           // -1 for the upper member, 0 otherwise
    x = p + ((x ^ neg) - neg);
  }
}

template <int CTRL, bool MAD24>
__device__ __forceinline__ void lane_bfly(uint32_t& x, int32_t sgn) {
  int32_t v = (int32_t)x;
  lane_bfly<CTRL, MAD24>(v, sgn);
  x = (uint32_t)v;
}

template <int CTRL, bool MAD24>
__device__ __forceinline__ void lane_bfly(double& x, int32_t sgn) {
  const uint64_t u = __double_as_longlong(x);
  const int32_t lo = __builtin_amdgcn_mov_dpp((int32_t)(uint32_t)u, CTRL, 0xF, 0xF, true);
  const int32_t hi = __builtin_amdgcn_mov_dpp((int32_t)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
  const double p = __longlong_as_double(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  x = fma(x, (double)sgn, p);                // exact: sgn = +-1
}

// Per-lane signs of the NL lane stages (see wht_lanes for directions and masks).
template <int NL>
__device__ __forceinline__ void lane_signs(int lam, int32_t* sg) {
  constexpr int um[4][4] = {{1, 0, 0, 0}, {1, 2, 0, 0}, {4, 5, 6, 0}, {8, 12, 5, 6}};
#pragma unroll
  for (int k = 0; k < NL; ++k) {
    sg[k] = (__popc((unsigned)(lam & um[NL > 0 ? NL - 1 : 0][k])) & 1) ? -1 : 1;
    asm volatile("" : "+v"(sg[k]));          // keep the +-1 range opaque (see lane_stage)
  }
}

template <int NL, bool MAD24, typename T>
__device__ __forceinline__ void wht_lanes1(T& x, const int32_t* sg) {
  if constexpr (NL == 1) {
    lane_bfly<kDppQuadXor1, MAD24>(x, sg[0]);
  } else if constexpr (NL == 2) {
    lane_bfly<kDppQuadXor1, MAD24>(x, sg[0]);
    lane_bfly<kDppQuadXor2, MAD24>(x, sg[1]);
  } else if constexpr (NL == 3) {
    lane_bfly<kDppHalfMirror, MAD24>(x, sg[0]);
    lane_bfly<kDppQuadXor1, MAD24>(x, sg[1]);
    lane_bfly<kDppQuadXor2, MAD24>(x, sg[2]);
  } else if constexpr (NL == 4) {
    lane_bfly<kDppMirror, MAD24>(x, sg[0]);
    lane_bfly<kDppHalfMirror, MAD24>(x, sg[1]);
    lane_bfly<kDppQuadXor1, MAD24>(x, sg[2]);
    lane_bfly<kDppQuadXor2, MAD24>(x, sg[3]);
  }
}

// wht_lanes1 on N independent values, stage by stage, so that the DPP moves of the N
// chains interleave (no wait states between a stage and the next).
template <int NL, bool MAD24, int N, typename T>
__device__ __forceinline__ void wht_lanes_n(T* x, const int32_t* sg) {
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if constexpr (NL == 1) lane_bfly<kDppQuadXor1, MAD24>(x[j], sg[0]);
    if constexpr (NL == 2) lane_bfly<kDppQuadXor1, MAD24>(x[j], sg[0]);
    if constexpr (NL == 3) lane_bfly<kDppHalfMirror, MAD24>(x[j], sg[0]);
    if constexpr (NL == 4) lane_bfly<kDppMirror, MAD24>(x[j], sg[0]);
  }
  if constexpr (NL >= 2) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if constexpr (NL == 2) lane_bfly<kDppQuadXor2, MAD24>(x[j], sg[1]);
      if constexpr (NL == 3) lane_bfly<kDppQuadXor1, MAD24>(x[j], sg[1]);
      if constexpr (NL == 4) lane_bfly<kDppHalfMirror, MAD24>(x[j], sg[1]);
    }
  }
  if constexpr (NL >= 3) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if constexpr (NL == 3) lane_bfly<kDppQuadXor2, MAD24>(x[j], sg[2]);
      if constexpr (NL == 4) lane_bfly<kDppQuadXor1, MAD24>(x[j], sg[2]);
    }
  }
  if constexpr (NL >= 4) {
#pragma unroll
    for (int j = 0; j < N; ++j) lane_bfly<kDppQuadXor2, MAD24>(x[j], sg[3]);
  }
}

// Sum of a 32-bit value over the 2^NL lanes of a row group (result valid in every lane).
template <int NL>
__device__ __forceinline__ uint32_t lane_sum(uint32_t x) {
  if constexpr (NL >= 4) x += (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kDppMirror, 0xF, 0xF, true);
  if constexpr (NL >= 3) x += (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kDppHalfMirror, 0xF, 0xF, true);
  if constexpr (NL >= 2) x += (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kDppQuadXor2, 0xF, 0xF, true);
  if constexpr (NL >= 1) x += (uint32_t)__builtin_amdgcn_mov_dpp((int)x, kDppQuadXor1, 0xF, 0xF, true);
  return x;
}

template <int Q>
struct StreamGeom {
  static constexpr int V = Q >= 3 ? 8 : (1 << Q);  // outcomes per lane
  static constexpr int LB = ilog2c(V);              // qubits folded in registers
  static constexpr int LPC = (1 << Q) / V;          // lanes per tile row
  static constexpr int LL = Q - LB;                 // outcome bits across lanes
  static constexpr int NSEQ = (int)ipow3(LB);       // rows walked by one lane group
  static constexpr int NRS = (int)ipow3(Q - LB);    // row-sets (walks) per tile
  static constexpr int NACC = (int)ipow4(Q);
  static constexpr int NROWS = (int)ipow3(Q);
};

// LDS slot of Pauli index a: [letters of the LB register qubits][letters of the lane
// qubits], the lane letters XOR-swizzled by the register letters.  An emission (one
// register-letter code for the whole wave, lane letters differing) and the write-out
// (consecutive a, i.e. consecutive register letters) both spread over the banks.
// For 4 lane qubits the top letter (bits 6-7) is also folded into the low bits (a
// bijection), which spreads the 16 lanes of a group and the 4 groups of a wave over
// more banks (fewer passes per binary64 atomic; modelled on the host).
// Both maps below are linear over XOR (for u < 256, (u >> 6) * 9 = h | h << 3 with
// h = u >> 6 only touches bits 0-4), so the slot splits as
//   slot = slot_fold(alane) ^ slot_key(areg):
// the lane part is set once per row-set and every emission (areg a compile-time
// constant, or a constant XOR one runtime digit) costs one XOR.
template <int Q, int LB>
__host__ __device__ constexpr uint32_t slot_fold(uint32_t u) {
  if constexpr (Q - LB == 4) return u ^ ((u >> 6) * 9u);
  else return u;
}

template <int Q, int LB>
__host__ __device__ constexpr uint32_t slot_key(uint32_t areg) {
  constexpr uint32_t hmask = (1u << (2 * (Q - LB))) - 1;
  return (areg << (2 * (Q - LB))) ^ slot_fold<Q, LB>(areg & hmask);
}

template <int Q, int LB>
__host__ __device__ constexpr uint32_t stream_slot_of(uint32_t areg, uint32_t alane) {
  return slot_fold<Q, LB>(alane) ^ slot_key<Q, LB>(areg);
}

template <int Q, int LB>
__host__ __device__ constexpr uint32_t stream_slot(uint32_t a) {
  return stream_slot_of<Q, LB>(a & ((1u << (2 * LB)) - 1), a >> (2 * LB));
}

// One block of the counts pass: block index `blk` -> (b_hi, run of `chunks` s_hi tiles).
// acc / rs_acc: LDS of NACC accumulators and NROWS row totals.  Every thread of the
// block calls this (it synchronises the block).
template <int Q, int THREADS, typename Acc, bool PER_BASIS, Out MODE, bool MAD24, bool PREFETCH = PER_BASIS>
// check_flags (blocks that cover whole rows, i.e. chunks == 2^(n-Q)): check the row
// totals in the block, against `shots` or the per-basis totals check_nb, instead of
// writing rowpart.
__device__ __forceinline__ void counts_block(const uint16_t* __restrict__ counts, int n, int chunks,
                                             const double* __restrict__ inv_nb, void* __restrict__ out,
                                             uint32_t* __restrict__ rowpart, uint64_t shots, int64_t blk,
                                             int tid, Acc* __restrict__ acc, uint32_t* __restrict__ rs_acc,
                                             uint32_t* __restrict__ check_flags = nullptr,
                                             const uint32_t* __restrict__ check_nb = nullptr, int lrow = -1) {
  using G = StreamGeom<Q>;
  constexpr int GROUPS = THREADS / G::LPC;
  constexpr int LB = G::LB;

  const int grp = tid / G::LPC, lam = tid % G::LPC;
  const int64_t n_shi = (int64_t)1 << (n - Q);
  const int64_t runs_per_row = n_shi / chunks;
  const int64_t b_hi = blk / runs_per_row;
  const int64_t s_hi0 = (blk % runs_per_row) * chunks;
  const int64_t row0 = b_hi * G::NROWS;
  // lrow: log2 of the row stride in counts (n unless the tile reads a segment of longer
  // rows, as a streamed slab does)
  const int64_t rowlen = (int64_t)1 << (lrow < 0 ? n : lrow);

  int32_t sg[G::LL > 0 ? G::LL : 1];
  lane_signs<G::LL>(lam, sg);
  const int lw = lane_walsh<G::LL>(lam);

  for (int i = tid; i < G::NACC; i += THREADS) acc[i] = Acc(0);
  for (int i = tid; i < G::NROWS; i += THREADS) rs_acc[i] = 0;
  __syncthreads();

  // Letters of the lane qubits for this lane's (relabelled) Walsh index in row-set rs:
  // the low bits of the LDS slot.
  auto ulane_of = [&](int rs) __attribute__((always_inline)) {
    uint32_t u = 0;
    int t = rs;
#pragma unroll
    for (int j = 0; j < G::LL; ++j) {
      if ((lw >> j) & 1) u += (uint32_t)(t % 3 + 1) << (2 * j);
      t /= 3;
    }
    return u;
  };

  // Carry: every group walks the same number of steps, so the prefetch issued by a
  // group's last step of one tile can fetch its first step of the next tile (same rows,
  // the next 2^Q outcomes): the loads stay in flight across the write-out.  With an odd
  // step count that prefetch lands in the second buffer and moves to the first one at
  // the next tile.
  constexpr bool kCarry = LB == 3 && PREFETCH && G::NRS % GROUPS == 0;
  constexpr bool kOddSteps = ((3 * G::NRS / GROUPS) & 1) == 1;
  uint32_t bufA[9][4], bufB[9][4];
  double invA = 0.0, invB = 0.0;

  for (int c = 0; c < chunks; ++c) {
    const int64_t s_hi = s_hi0 + c;
    const uint16_t* __restrict__ cchunk = counts + row0 * rowlen + (s_hi << Q) + lam * G::V;
    if constexpr (LB == 3) {
      // A step is 9 rows (basis digits d0, d1 of qubits 0, 1) at fixed d2 of row-set rs;
      // a group walks steps (rs, 0), (rs, 1), (rs, 2), (rs + GROUPS, 0), ...
      Acc L1[4][2], L2[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a) { L1[a][0] = L1[a][1] = Acc(0); L2[a][0] = L2[a][1] = L2[a][2] = L2[a][3] = Acc(0); }
      uint32_t ubase = 0;   // slot_fold(lane letters) * sizeof(Acc): byte offset of the lane part
      // dummy: a prefetch past the group's last step reads the tile's first row segment
      // nine times (cached) instead of fresh rows.
      // next_tile: rows of step (rs, d2) in the next tile (2^Q outcomes further on).
      auto load9 = [&](uint32_t (&buf)[9][4], double& invr, int rs, int d2, bool dummy = false,
                       bool next_tile = false) __attribute__((always_inline)) {
        const int rr = dummy ? 0 : rs * G::NSEQ + 9 * d2;
        const uint16_t* __restrict__ p = cchunk + (int64_t)rr * rowlen + (next_tile ? (1 << Q) : 0);
        const int64_t stride = dummy ? 0 : rowlen;
#pragma unroll
        for (int r = 0; r < 9; ++r) load_raw<8>(p + (int64_t)r * stride, buf[r]);
        if constexpr (PER_BASIS && G::LPC >= 9) invr = inv_nb[row0 + rr + (lam < 9 ? lam : 0)];  // lane r: row r
      };
      // Four emissions at once: lane butterflies interleaved, then the four LDS adds.
      // base: ubase, possibly XORed with the key of a runtime digit; areg: constants.
      auto emit4 = [&](Acc (&v)[4], const uint32_t (&areg)[4], uint32_t base) __attribute__((always_inline)) {
        wht_lanes_n<G::LL, MAD24, 4>(v, sg);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          atomicAdd(reinterpret_cast<Acc*>(reinterpret_cast<char*>(acc) +
                                           (base ^ (slot_key<Q, LB>(areg[j]) * (uint32_t)sizeof(Acc)))),
                    v[j]);
      };
      // first: the group's first step (its row-set's letters are not yet set up);
      // last: the group's last step (flush the qubit-2 identity sums even mid row-set).
      auto step = [&](const uint32_t (&raw)[9][4], double invr, int rs, int d2, bool first,
                      bool last) __attribute__((always_inline)) {
        if (first || d2 == 0) ubase = slot_fold<Q, LB>(ulane_of(rs)) * (uint32_t)sizeof(Acc);
        const int rr = rs * G::NSEQ + 9 * d2;
        // Letter d2 + 1 of qubit 2 (bits 4-5 of the register letters) in every emission
        // of this step except the qubit-2 identity ones.
        const uint32_t b2 = ubase ^ (slot_key<Q, LB>(16u * (uint32_t)(d2 + 1)) * (uint32_t)sizeof(Acc));
        StaticFor<0, 3>::run([&](auto d1c) __attribute__((always_inline)) {
          constexpr int d1 = decltype(d1c)::value;
          Acc L0[4] = {Acc(0), Acc(0), Acc(0), Acc(0)};
          Acc pend[4];   // the (X/Y/Z, X/Y/Z, X/Y/Z) value of each of the 3 rows, then L0's
          StaticFor<0, 3>::run([&](auto d0c) __attribute__((always_inline)) {
            constexpr int d0 = decltype(d0c)::value;
            constexpr int r = 3 * d1 + d0;
            int32_t x[8];
            unpack_raw<8>(raw[r], x);
            wht_regs<3>(x);
            const uint32_t tot = lane_sum<G::LL>((uint32_t)x[0]);
            if (lam == 0) atomicAdd(&rs_acc[rr + r], tot);
            Acc y[8];
            if constexpr (PER_BASIS) {
              // 1/N_b of row r: held by lane r of the group (16 lanes), else loaded here.
              double inv;
              if constexpr (G::LPC >= 9) inv = __shfl(invr, (tid & 63 & ~(G::LPC - 1)) + r, 64);
              else inv = inv_nb[row0 + rr + r];
#pragma unroll
              for (int v = 0; v < 8; ++v) y[v] = (double)x[v] * inv;
            } else {
#pragma unroll
              for (int v = 0; v < 8; ++v) y[v] = to_acc<Acc>(x[v]);
            }
            // y[v], v = m0 + 2 m1 + 4 m2.  Qubit 0: m0 = 0 -> identity (L0); m0 = 1 -> letter d0+1.
#pragma unroll
            for (int mr = 0; mr < 4; ++mr) {
              L0[mr] += y[2 * mr];
              const Acc w = y[2 * mr + 1];
              const int m1 = mr & 1, m2 = mr >> 1;
              if (m1 == 0) L1[d0 + 1][m2] += w;
              else if (m2 == 0) L2[d0 + 1][d1 + 1] += w;
              else pend[d0] = w;
            }
          });
          // End of the qubit-0 walk: its identity sums move up (letter I at qubit 0).
#pragma unroll
          for (int mr = 0; mr < 4; ++mr) {
            const int m1 = mr & 1, m2 = mr >> 1;
            if (m1 == 0) L1[0][m2] += L0[mr];
            else if (m2 == 0) L2[0][d1 + 1] += L0[mr];
            else pend[3] = L0[mr];
          }
          const uint32_t ar[4] = {1u + 4u * (d1 + 1), 2u + 4u * (d1 + 1), 3u + 4u * (d1 + 1), 4u * (d1 + 1)};
          emit4(pend, ar, b2);
        });
        // End of the qubit-1 walk (letters of qubit 1 now final).
        {
          Acc v1[4];
          const uint32_t ar[4] = {0u, 1u, 2u, 3u};
#pragma unroll
          for (int a0 = 0; a0 < 4; ++a0) {
            L2[a0][0] += L1[a0][0];
            v1[a0] = L1[a0][1];
            L1[a0][0] = L1[a0][1] = Acc(0);
          }
          emit4(v1, ar, b2);
        }
        if (d2 == 2 || last) {
          // End of the qubit-2 walk (or of this group's part of it): identity letter at qubit 2.
#pragma unroll
          for (int a1 = 0; a1 < 4; ++a1) {
            Acc v2[4] = {L2[0][a1], L2[1][a1], L2[2][a1], L2[3][a1]};
            const uint32_t ar[4] = {0u + 4u * a1, 1u + 4u * a1, 2u + 4u * a1, 3u + 4u * a1};
            emit4(v2, ar, ubase);
#pragma unroll
            for (int a0 = 0; a0 < 4; ++a0) L2[a0][a1] = Acc(0);
          }
        }
      };
      // Steps are numbered s = 3 rs + d2 (243 per tile for Q = 7); group g takes the
      // steps of a contiguous range of whole row-sets, so that the groups of a wave reach
      // the end of a row-set together.  (The step loop also handles a range that starts
      // or ends inside a row-set: the qubit-2 identity sums are then flushed as partial
      // sums, which the LDS adds.)
      const int s0 = 3 * (int)(((int64_t)grp * G::NRS) / GROUPS);
      const int s1 = 3 * (int)(((int64_t)(grp + 1) * G::NRS) / GROUPS);
      if constexpr (PREFETCH) {
        // Double-buffered: the next step's rows are in flight while this one is folded.
        // The prefetch is unconditional (past the last step it is a cached dummy read) so
        // that the wait for the current buffer never has to cover it.
        if constexpr (kCarry) {
          // NST steps per group, known at compile time, so the buffer that receives the
          // next tile's rows is known statically too.
          constexpr int NST = 3 * G::NRS / GROUPS;
          const bool carry = c + 1 < chunks;   // else the last prefetch is a dummy
          if (c == 0) {
            load9(bufA, invA, s0 / 3, s0 % 3);
          } else if constexpr (kOddSteps) {
#pragma unroll
            for (int r = 0; r < 9; ++r)
#pragma unroll
              for (int k = 0; k < 4; ++k) bufA[r][k] = bufB[r][k];
            invA = invB;
          }
          int s = s0;
#pragma unroll 1
          for (int i = 0; i + 1 < NST; i += 2) {
            load9(bufB, invB, (s + 1) / 3, (s + 1) % 3);
            step(bufA, invA, s / 3, s % 3, i == 0, false);
            ++s;
            const bool more = i + 2 < NST;
            const int sn = more ? s + 1 : s0;
            load9(bufA, invA, sn / 3, sn % 3, !more && !carry, !more && carry);
            step(bufB, invB, s / 3, s % 3, false, !more);
            ++s;
          }
          if constexpr (kOddSteps) {
            load9(bufB, invB, s0 / 3, s0 % 3, !carry, carry);
            step(bufA, invA, s / 3, s % 3, NST == 1, true);
          }
        } else if (s0 < s1) {
          int s = s0;
          load9(bufA, invA, s / 3, s % 3);
          for (;;) {
            int sn = s + 1;
            bool more = sn < s1;
            load9(bufB, invB, sn / 3, sn % 3, !more);
            step(bufA, invA, s / 3, s % 3, s == s0, !more);
            if (!more) break;
            s = sn;
            sn = s + 1;
            more = sn < s1;
            load9(bufA, invA, sn / 3, sn % 3, !more);
            step(bufB, invB, s / 3, s % 3, false, !more);
            if (!more) break;
            s = sn;
          }
        }
      } else {
#pragma unroll 1
        for (int s = s0; s < s1; ++s) {
          uint32_t raw[9][4];
          double invr = 0.0;
          load9(raw, invr, s / 3, s % 3);
          step(raw, invr, s / 3, s % 3, s == s0, s + 1 == s1);
        }
      }
    } else {
      // Small tiles (Q < 3): one lane holds a whole row (LPC = 1); plain direct fold.
      static_assert(G::LPC == 1, "small-tile path expects one lane per row");
      for (int rs = grp; rs < G::NRS; rs += GROUPS) {
        const int64_t rowb = row0 + (int64_t)rs * G::NSEQ;
        for (int r = 0; r < G::NSEQ; ++r) {
          uint32_t raw[G::V / 2];
          load_raw<G::V>(cchunk + (int64_t)(rs * G::NSEQ + r) * rowlen, raw);
          int32_t x[G::V];
          unpack_raw<G::V>(raw, x);
          wht_regs<LB>(x);
          atomicAdd(&rs_acc[rs * G::NSEQ + r], (uint32_t)x[0]);
          double inv = 1.0;
          if constexpr (PER_BASIS) inv = inv_nb[rowb + r];
#pragma unroll
          for (int m = 0; m < G::V; ++m) {
            uint32_t areg = 0;
            int t = r;
#pragma unroll
            for (int k = 0; k < LB; ++k) {
              if ((m >> k) & 1) areg += (uint32_t)(t % 3 + 1) << (2 * k);
              t /= 3;
            }
            Acc v;
            if constexpr (PER_BASIS) v = (double)x[m] * inv;
            else v = to_acc<Acc>(x[m]);
            atomicAdd(&acc[stream_slot_of<Q, LB>(areg, 0)], v);
          }
        }
      }
    }
    lds_barrier();   // the carried prefetch stays in flight across the write-out

    for (int i = tid; i < G::NACC; i += THREADS) {
      const uint32_t slot = stream_slot<Q, LB>((uint32_t)i);
      const Acc v = acc[slot];
      acc[slot] = Acc(0);
      if constexpr (MODE == Out::Partial) {
        // Partials are re-read only by the next pass, far beyond what the caches hold.
        __builtin_nontemporal_store(v, &static_cast<Acc*>(out)[(b_hi * n_shi + s_hi) * G::NACC + i]);
      } else if constexpr (MODE == Out::CoefUniform) {
        const int w = pauli_weight((uint64_t)i);
        static_cast<double*>(out)[i] = acc_to_double(v) / (pow3d(n - w) * (double)shots);
      } else if constexpr (MODE == Out::CoefPerBasis) {
        const int w = pauli_weight((uint64_t)i);
        static_cast<double*>(out)[i] = acc_to_double(v) / pow3d(n - w);
      } else {
        static_cast<int64_t*>(out)[i] = acc_to_i64(v);
      }
    }
    lds_barrier();
  }

  if (check_flags) {
    // The block covered every outcome of its rows: check the totals here, against the
    // uniform shots or (check_nb) the per-basis totals.
    for (int i = tid; i < G::NROWS; i += THREADS) {
      const uint32_t want = check_nb ? check_nb[row0 + i] : (uint32_t)shots;
      if (rs_acc[i] != want) atomicOr(check_flags, (uint32_t)FLAG_SHOTS);
    }
  } else {
    uint32_t* __restrict__ rp = rowpart + blk * G::NROWS;
    for (int i = tid; i < G::NROWS; i += THREADS) rp[i] = rs_acc[i];
  }
}

template <int Q, int THREADS, typename Acc, bool PER_BASIS, Out MODE, bool MAD24, int MINWAVES = 1,
          bool PREFETCH = PER_BASIS>
__global__ __launch_bounds__(THREADS, MINWAVES) void fold_counts_stream_kernel(
    const uint16_t* __restrict__ counts, int n, int chunks, const double* __restrict__ inv_nb,
    void* __restrict__ out, uint32_t* __restrict__ rowpart, uint64_t shots, int lrow) {
  __shared__ Acc acc[StreamGeom<Q>::NACC];
  __shared__ uint32_t rs_acc[StreamGeom<Q>::NROWS];
  counts_block<Q, THREADS, Acc, PER_BASIS, MODE, MAD24, PREFETCH>(counts, n, chunks, inv_nb, out, rowpart, shots,
                                                                 blockIdx.x, threadIdx.x, acc, rs_acc, nullptr,
                                                                 nullptr, lrow);
}

// ---------------------------------------------------------------------------------
// Counts pass on int8 MFMA (Q = 7 qubits per tile).  The Walsh-Hadamard transform over
// the low 6 outcome bits of every basis row is a dense +-1 contraction,
//   S[m][row] = sum_{s < 64} H64[m][s] c[row][s],
// run as v_mfma_i32_16x16x64_i8 with A = four 16-row blocks of H64 and B = counts.
// A uint16 count c = b0 + 256 b1 is fed as two signed byte limbs l0 = b0 - 128,
// l1 = b1 - 128 (c = l0 + 256 l1 + 32896); the constant 32896 only reaches Walsh row 0
// (the only row of H64 with a nonzero sum, 64), so
//   S = D(l0) + 256 D(l1) + 32896 * 64 * [m == 0]      exactly, in int32.
// Lane l of an MFMA holds B column n = l % 16 and 16 K slots; A row l % 16 with the same
// 16 K slots (the K order is internal to the instruction and common to A and B).  The
// result lane l holds rows 4 (l / 16) + r, r < 4, of column l % 16.
// Columns are 16 row-sets; the 3 rows of the lowest basis digit are 3 MFMA tiles in
// sequence, so the lowest qubit is folded in registers (and per-basis division by N_b
// happens per row before any cross-row sum).  Outcome bit 6 is a second 64-count block
// combined with one butterfly in registers.  The remaining 6 qubits are summed over
// basis letters in the LDS accumulator (atomics), as in the plain kernel.
typedef int lre_v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ lre_v4i limb_pack(const uint32_t* w, uint32_t sel) {
  lre_v4i o;
  o.x = (int)(__builtin_amdgcn_perm(w[1], w[0], sel) ^ 0x80808080u);
  o.y = (int)(__builtin_amdgcn_perm(w[3], w[2], sel) ^ 0x80808080u);
  o.z = (int)(__builtin_amdgcn_perm(w[5], w[4], sel) ^ 0x80808080u);
  o.w = (int)(__builtin_amdgcn_perm(w[7], w[6], sel) ^ 0x80808080u);
  return o;
}

// LDS slot of a Pauli index a (7 digits) in the MFMA counts-pass accumulator:
// [a_0][a_1][a_4][a_5][a_6][a_2][a_3] (most significant first) -- the digits that
// come from lane bits (positions 2, 3) are the low bits.
__device__ __forceinline__ uint32_t mfma_slot(uint32_t a) {
  const uint32_t d0 = a & 3, d1 = (a >> 2) & 3, d2 = (a >> 4) & 3, d3 = (a >> 6) & 3;
  const uint32_t d4 = (a >> 8) & 3, d5 = (a >> 10) & 3, d6 = (a >> 12) & 3;
  return (d0 << 12) | (d1 << 10) | (d4 << 8) | (d5 << 6) | (d6 << 4) | (d2 << 2) | d3;
}

// A operand of the 64-point transform for lane (g, col): rows 16 mb + col of H64, K slots
// 16 g + j, entries +-1 as int8.
__device__ __forceinline__ void mfma_h64_operand(int col, int g, lre_v4i (&hA)[4]) {
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const int m = 16 * mb + col;
    int wv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t wd = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int k = 16 * g + 4 * q + b;
        const uint32_t v = (__popc((unsigned)(m & k)) & 1) ? 0xFFu : 0x01u;
        wd |= v << (8 * b);
      }
      wv[q] = (int)wd;
    }
    hA[mb] = lre_v4i{wv[0], wv[1], wv[2], wv[3]};
  }
}

// Walsh-Hadamard transform of 64 outcomes on int8 MFMA, exact in int32: lane (g, col)
// supplies counts 16 g .. 16 g + 15 of column col's 64-outcome segment in w (uint16
// pairs) and receives S[mb][r], Walsh index 16 mb + 4 g + r of its column.  Two biased
// byte limbs per count (c = l0 + 256 l1 + 32896); the bias only reaches Walsh row 0.
__device__ __forceinline__ void mfma_wht64(const lre_v4i (&hA)[4], const uint32_t (&w)[8], int g,
                                           int32_t (&S)[4][4]) {
  const lre_v4i l0 = limb_pack(w, 0x06040200u);
  const lre_v4i l1 = limb_pack(w, 0x07050301u);
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    const lre_v4i z = {0, 0, 0, 0};
    const lre_v4i d0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(hA[mb], l0, z, 0, 0, 0);
    const lre_v4i d1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(hA[mb], l1, z, 0, 0, 0);
    S[mb][0] = d0.x + (d1.x << 8);
    S[mb][1] = d0.y + (d1.y << 8);
    S[mb][2] = d0.z + (d1.z << 8);
    S[mb][3] = d0.w + (d1.w << 8);
  }
  if (g == 0) S[0][0] += 32896 * 64;  // bias of the limb encoding (Walsh row 0)
}

template <int THREADS, typename Acc, bool PER_BASIS, Out MODE>
__global__ __launch_bounds__(THREADS) void fold_counts_mfma_kernel(
    const uint16_t* __restrict__ counts, int n, int chunks, const uint32_t* __restrict__ nb,
    void* __restrict__ out, uint32_t* __restrict__ rowpart, uint64_t shots, int lrow) {
  constexpr int Q = 7;
  constexpr int NACC = 1 << (2 * Q);
  constexpr int NROWS = 2187;   // 3^7
  constexpr int NRS = 729;      // row-sets of 3 rows
  constexpr int WAVES = THREADS / 64;
  __shared__ Acc acc[NACC];
  __shared__ uint32_t rs_acc[NROWS];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, g = lane >> 4;
  const int64_t n_shi = (int64_t)1 << (n - Q);
  const int64_t runs_per_row = n_shi / chunks;
  const int64_t b_hi = blockIdx.x / runs_per_row;
  const int64_t s_hi0 = (blockIdx.x % runs_per_row) * chunks;
  const int64_t row0 = b_hi * NROWS;
  const int64_t rowlen = (int64_t)1 << lrow;   // row stride (n, or more for a slab segment)

  lre_v4i hA[4];
  mfma_h64_operand(col, g, hA);

  for (int i = tid; i < NACC; i += THREADS) acc[i] = Acc(0);
  for (int i = tid; i < NROWS; i += THREADS) rs_acc[i] = 0;
  __syncthreads();

  for (int c = 0; c < chunks; ++c) {
    const int64_t s_hi = s_hi0 + c;
    for (int rs0 = wave * 16; rs0 < NRS; rs0 += WAVES * 16) {
      const int rs = rs0 + col;
      const bool valid = rs < NRS;
      // Basis digits of the row-set (positions 1..6) -> letter terms of the LDS slot.
      uint32_t t1, t2, t3, t4, t5, t6;
      {
        int t = valid ? rs : 0;
        t1 = (uint32_t)(t % 3 + 1) << 10; t /= 3;
        t2 = (uint32_t)(t % 3 + 1) << 2;  t /= 3;
        t3 = (uint32_t)(t % 3 + 1);       t /= 3;
        t4 = (uint32_t)(t % 3 + 1) << 8;  t /= 3;
        t5 = (uint32_t)(t % 3 + 1) << 6;  t /= 3;
        t6 = (uint32_t)(t % 3 + 1) << 4;
      }
      const uint32_t ulane = ((g & 1) ? t2 : 0u) + ((g & 2) ? t3 : 0u);

      Acc iacc[2][4][2];  // identity letter of qubit 0: [m6][mb][m1]
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) { iacc[a][b][0] = Acc(0); iacc[a][b][1] = Acc(0); }

#pragma unroll 1
      for (int beta = 0; beta < 3; ++beta) {
        const int64_t row = row0 + 3 * (int64_t)rs + beta;
        int32_t S[2][4][4];  // [outcome bit 6][mb][r]
#pragma unroll
        for (int sb = 0; sb < 2; ++sb) {
          uint32_t w[8];
          if (valid) {
            const uint4* p = reinterpret_cast<const uint4*>(counts + row * rowlen + (s_hi << Q) + 64 * sb + 16 * g);
            const uint4 u0 = p[0], u1 = p[1];
            w[0] = u0.x; w[1] = u0.y; w[2] = u0.z; w[3] = u0.w;
            w[4] = u1.x; w[5] = u1.y; w[6] = u1.z; w[7] = u1.w;
          } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) w[k] = 0;
          }
          mfma_wht64(hA, w, g, S[sb]);
        }
        // Butterfly on outcome bit 6: S[0] <- m6 = 0, S[1] <- m6 = 1.
#pragma unroll
        for (int mb = 0; mb < 4; ++mb)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int32_t a = S[0][mb][r], b = S[1][mb][r];
            S[0][mb][r] = a + b;
            S[1][mb][r] = a - b;
          }
        // Row total (Walsh index 0) for the row check.
        if (valid && g == 0) atomicAdd(&rs_acc[3 * rs + beta], (uint32_t)S[0][0][0]);

        double inv = 1.0;
        if constexpr (PER_BASIS) {
          const uint32_t N = valid ? nb[row] : 1u;
          inv = N ? 1.0 / (double)N : 0.0;  // empty basis: flagged by the row check
        }
        // Qubit 0: Walsh bit m0 = bit 0 of r.  m0 = 0 -> identity letter (sum over beta);
        // m0 = 1 -> letter beta + 1, final for this qubit: add to LDS now.
#pragma unroll
        for (int m6 = 0; m6 < 2; ++m6)
#pragma unroll
          for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int m1 = 0; m1 < 2; ++m1) {
              Acc v0, v1;
              if constexpr (PER_BASIS) {
                v0 = (double)S[m6][mb][2 * m1] * inv;
                v1 = (double)S[m6][mb][2 * m1 + 1] * inv;
              } else {
                v0 = to_acc<Acc>(S[m6][mb][2 * m1]);
                v1 = to_acc<Acc>(S[m6][mb][2 * m1 + 1]);
              }
              iacc[m6][mb][m1] += v0;
              if (valid) {
                const uint32_t slot = ulane + (m1 ? t1 : 0u) + ((mb & 1) ? t4 : 0u) +
                                      ((mb & 2) ? t5 : 0u) + (m6 ? t6 : 0u) +
                                      ((uint32_t)(beta + 1) << 12);
                atomicAdd(&acc[slot], v1);
              }
            }
      }
      if (valid) {
#pragma unroll
        for (int m6 = 0; m6 < 2; ++m6)
#pragma unroll
          for (int mb = 0; mb < 4; ++mb)
#pragma unroll
            for (int m1 = 0; m1 < 2; ++m1) {
              const uint32_t slot = ulane + (m1 ? t1 : 0u) + ((mb & 1) ? t4 : 0u) +
                                    ((mb & 2) ? t5 : 0u) + (m6 ? t6 : 0u);
              atomicAdd(&acc[slot], iacc[m6][mb][m1]);
            }
      }
    }
    __syncthreads();

    for (int i = tid; i < NACC; i += THREADS) {
      const uint32_t slot = mfma_slot((uint32_t)i);
      const Acc v = acc[slot];
      acc[slot] = Acc(0);
      if constexpr (MODE == Out::Partial) {
        static_cast<Acc*>(out)[(b_hi * n_shi + s_hi) * NACC + i] = v;
      } else if constexpr (MODE == Out::CoefUniform) {
        const int w = pauli_weight((uint64_t)i);
        static_cast<double*>(out)[i] = acc_to_double(v) / (pow3d(n - w) * (double)shots);
      } else if constexpr (MODE == Out::CoefPerBasis) {
        const int w = pauli_weight((uint64_t)i);
        static_cast<double*>(out)[i] = acc_to_double(v) / pow3d(n - w);
      } else {
        static_cast<int64_t*>(out)[i] = acc_to_i64(v);
      }
    }
    __syncthreads();
  }

  uint32_t* __restrict__ rp = rowpart + (int64_t)blockIdx.x * NROWS;
  for (int i = tid; i < NROWS; i += THREADS) rp[i] = rs_acc[i];
}

// ---------------------------------------------------------------------------------
// Later passes: [3^h][2^h][4^l] -> [3^{h-F}][2^{h-F}][4^{F+l}], one thread per column
// (b_hi, s_hi, a_lo), a_lo fastest so that loads and stores are coalesced.

template <typename Tin, typename Acc>
__device__ __forceinline__ Acc in_to_acc(Tin v) {
  if constexpr (sizeof(Tin) == 4 && sizeof(Acc) == 4) return (Acc)(uint32_t)v;
  else if constexpr (sizeof(Tin) == 4) return (Acc)(int32_t)(uint32_t)v;
  else return (Acc)v;
}

// Input element (beta, sg) of column `col` in a later pass: beta = basis digits and
// sg = outcome bits of the F qubits being folded.
template <int F>
__device__ __forceinline__ int64_t fold_in_offset(int h, int l, int64_t col, int beta, int sg) {
  const int64_t L = (int64_t)1 << (2 * l);
  const int64_t a_l = col & (L - 1);
  const int64_t bs = col >> (2 * l);
  const int hr = h - F;
  const int64_t s_hi = bs & (((int64_t)1 << hr) - 1);
  const int64_t b_hi = bs >> hr;
  const int64_t rowstride = ((int64_t)1 << h) * L;
  return (b_hi * ipow3(F) + beta) * rowstride + ((s_hi << F) + sg) * L + a_l;
}

// One column of a later pass: folds F more qubits of the partial tensor for the
// fastest-varying index column `col` (one thread per column, all in registers).
// src(beta, sg) returns input element (beta, sg) of the column as Tin.
template <int F, typename Tin, typename Acc, Out MODE, class Src>
__device__ __forceinline__ void fold_partial_col_src(Src&& src, void* __restrict__ out, int n, int h, int l,
                                                     uint64_t shots, int64_t col) {
  const int64_t L = (int64_t)1 << (2 * l);
  const int64_t a_l = col & (L - 1);
  const int64_t bs = col >> (2 * l);

  constexpr int NA = (int)ipow4(F);
  // Final value of folded letter code a (compile-time) for this column.  The divisor
  // depends on the weight only through the k <= F new non-identity letters: den[k].
  const int wl = MODE == Out::Partial ? 0 : pauli_weight((uint64_t)a_l);
  double den[F + 1];
  if constexpr (MODE == Out::CoefUniform || MODE == Out::CoefPerBasis) {
#pragma unroll
    for (int k = 0; k <= F; ++k)
      den[k] = MODE == Out::CoefUniform ? pow3d(n - wl - k) * (double)shots : pow3d(n - wl - k);
  }
  auto put = [&](auto ac, Acc v) __attribute__((always_inline)) {
    constexpr int a = decltype(ac)::value;
    if constexpr (MODE == Out::Partial) {
      static_cast<Acc*>(out)[bs * (NA * L) + a * L + a_l] = v;
    } else {
      const int64_t i = a * L + a_l;
      constexpr int k = __builtin_popcount((a | (a >> 1)) & 0x55555555);
      if constexpr (MODE == Out::CoefUniform || MODE == Out::CoefPerBasis)
        static_cast<double*>(out)[i] = acc_to_double(v) / den[k];
      else
        static_cast<int64_t*>(out)[i] = acc_to_i64(v);
    }
  };
  auto load_row = [&](int beta, Acc* x) __attribute__((always_inline)) {
#pragma unroll
    for (int sg = 0; sg < (1 << F); ++sg) x[sg] = in_to_acc<Tin, Acc>(src(beta, sg));
    wht_regs<F>(x);
  };
  using I0 = std::integral_constant<int, 0>;

  if constexpr (F == 3) {
    // Accumulator cascade over the basis digits (d0 innermost): level k holds the
    // identity-letter sums of position k; a letter code is stored as soon as it is final.
    Acc L1[4][2], L2[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) { L1[q][0] = L1[q][1] = Acc(0); L2[q][0] = L2[q][1] = L2[q][2] = L2[q][3] = Acc(0); }
    StaticFor<0, 3>::run([&](auto d2c) __attribute__((always_inline)) {
      constexpr int d2 = decltype(d2c)::value;
      StaticFor<0, 3>::run([&](auto d1c) __attribute__((always_inline)) {
        constexpr int d1 = decltype(d1c)::value;
        Acc L0[4] = {Acc(0), Acc(0), Acc(0), Acc(0)};
        StaticFor<0, 3>::run([&](auto d0c) __attribute__((always_inline)) {
          constexpr int d0 = decltype(d0c)::value;
          Acc y[8];
          load_row(d0 + 3 * d1 + 9 * d2, y);
          StaticFor<0, 4>::run([&](auto mrc) __attribute__((always_inline)) {
            constexpr int mr = decltype(mrc)::value, m1 = mr & 1, m2 = mr >> 1;
            L0[mr] += y[2 * mr];
            if constexpr (m1 == 0) L1[d0 + 1][m2] += y[2 * mr + 1];
            else if constexpr (m2 == 0) L2[d0 + 1][d1 + 1] += y[2 * mr + 1];
            else put(std::integral_constant<int, (d0 + 1) + 4 * (d1 + 1) + 16 * (d2 + 1)>{}, y[2 * mr + 1]);
          });
        });
        StaticFor<0, 4>::run([&](auto mrc) __attribute__((always_inline)) {
          constexpr int mr = decltype(mrc)::value, m1 = mr & 1, m2 = mr >> 1;
          if constexpr (m1 == 0) L1[0][m2] += L0[mr];
          else if constexpr (m2 == 0) L2[0][d1 + 1] += L0[mr];
          else put(std::integral_constant<int, 4 * (d1 + 1) + 16 * (d2 + 1)>{}, L0[mr]);
        });
      });
      StaticFor<0, 4>::run([&](auto a0c) __attribute__((always_inline)) {
        constexpr int a0 = decltype(a0c)::value;
        L2[a0][0] += L1[a0][0];
        put(std::integral_constant<int, a0 + 16 * (d2 + 1)>{}, L1[a0][1]);
        L1[a0][0] = L1[a0][1] = Acc(0);
      });
    });
    StaticFor<0, 16>::run([&](auto ac) __attribute__((always_inline)) {
      constexpr int a = decltype(ac)::value;
      put(ac, L2[a & 3][a >> 2]);
    });
  } else {
    Acc acc[NA];
    StaticFor<0, NA>::run([&](auto ac) __attribute__((always_inline)) { acc[decltype(ac)::value] = Acc(0); });
    StaticFor<0, (int)ipow3(F)>::run([&](auto bc) __attribute__((always_inline)) {
      constexpr int beta = decltype(bc)::value;
      Acc x[1 << F];
      load_row(beta, x);
      StaticFor<0, (1 << F)>::run([&](auto mc) __attribute__((always_inline)) {
        constexpr int m = decltype(mc)::value;
        constexpr int a = fold_index(beta, m, F);
        acc[a] += x[m];
      });
    });
    StaticFor<0, NA>::run([&](auto ac) __attribute__((always_inline)) { put(ac, acc[decltype(ac)::value]); });
  }
  (void)sizeof(I0);
}

template <int F, typename Tin, typename Acc, Out MODE>
__device__ __forceinline__ void fold_partial_col(const Tin* __restrict__ in, void* __restrict__ out, int n,
                                                 int h, int l, uint64_t shots, int64_t col) {
  const int64_t L = (int64_t)1 << (2 * l);
  const int64_t rowstride = ((int64_t)1 << h) * L;
  const Tin* __restrict__ p0 = in + fold_in_offset<F>(h, l, col, 0, 0);
  fold_partial_col_src<F, Tin, Acc, MODE>(
      [&](int beta, int sg) __attribute__((always_inline)) { return p0[beta * rowstride + sg * L]; }, out, n, h,
      l, shots, col);
}

template <int F, typename Tin, typename Acc, Out MODE>
__global__ __launch_bounds__(256) void fold_partial_kernel(const Tin* __restrict__ in,
                                                           void* __restrict__ out, int n, int h,
                                                           int l, uint64_t shots, int64_t ncols) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (col < ncols) fold_partial_col<F, Tin, Acc, MODE>(in, out, n, h, l, shots, col);
}

// Later pass folding 4 qubits (partials only): [3^h][2^h][4^l] -> [3^{h-4}][2^{h-4}][4^{4+l}].
// The 6^4 = 1296 inputs of a column do not fit one thread's registers, so a group of
// kF4Cols consecutive columns a_l of one outer index (b_hi, s_hi) keeps the 4^4 letter
// codes of each column in LDS.  Each of the block's kF4Waves waves takes 81 / kF4Waves
// of the basis-digit combinations beta, transforms the 16 outcome values of its column
// in registers (4-bit Walsh-Hadamard) and adds value m into letter code
// fold_index(beta, m); the identity letters collect their sums over beta through the
// LDS atomics.  Loads and stores are coalesced along a_l.  Blocks are persistent (one
// per LDS-sized slot of the device) and walk groups g, g + gridDim.x, ...: the next
// beta is loaded while the current one is folded, and a wave's last load of a group
// fetches its first beta of the next group, which stays in flight across the
// write-out (LDS-only barriers).
constexpr int kF4Cols = 64;
constexpr int kF4Waves = 9;

template <typename Tin, typename Acc>
__global__ __launch_bounds__(64 * kF4Waves) void fold_partial4_kernel(const Tin* __restrict__ in,
                                                                      Acc* __restrict__ out, int h, int l) {
  constexpr int NS = 16, NA = 256, PER = 81 / kF4Waves, TH = 64 * kF4Waves;
  static_assert(81 % kF4Waves == 0 && PER % 2 == 1, "waves split the 81 combinations into odd counts");
  __shared__ Acc acc[NA * kF4Cols];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t L = (int64_t)1 << (2 * l);
  const int64_t per_outer = L / kF4Cols;
  const int hr = h - 4;
  const int64_t total = (ipow3(hr) << hr) * per_outer;
  const int64_t rowstride = ((int64_t)1 << h) * L;
  // First input of group g for this lane; the group's outer index and first column.
  auto group_in = [&](int64_t g) __attribute__((always_inline)) {
    const int64_t bs = g / per_outer, c0 = (g % per_outer) * kF4Cols;
    const int64_t s_hi = bs & (((int64_t)1 << hr) - 1), b_hi = bs >> hr;
    return in + b_hi * 81 * rowstride + (s_hi << 4) * L + c0 + lane;
  };
  // The loads are issued where they stand (the scheduler would otherwise sink them
  // below the transform of the previous buffer and the prefetch would not overlap it).
  auto load = [&](const Tin* __restrict__ p0, int beta, Acc (&x)[NS]) __attribute__((always_inline)) {
    const Tin* __restrict__ p = p0 + beta * rowstride;
#pragma unroll
    for (int sg = 0; sg < NS; ++sg) x[sg] = in_to_acc<Tin, Acc>(__builtin_nontemporal_load(&p[sg * L]));
    __builtin_amdgcn_sched_barrier(0);
  };
  auto fold = [&](int beta, Acc (&x)[NS]) __attribute__((always_inline)) {
    wht_regs<4>(x);
    const uint32_t t0 = (uint32_t)(beta % 3 + 1), t1 = (uint32_t)((beta / 3) % 3 + 1) << 2;
    const uint32_t t2 = (uint32_t)((beta / 9) % 3 + 1) << 4, t3 = (uint32_t)(beta / 27 + 1) << 6;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const uint32_t a = ((m & 1) ? t0 : 0u) | ((m & 2) ? t1 : 0u) | ((m & 4) ? t2 : 0u) | ((m & 8) ? t3 : 0u);
      atomicAdd(&acc[a * kF4Cols + lane], x[m]);
    }
  };

  for (int i = tid; i < NA * kF4Cols; i += TH) acc[i] = Acc(0);
  __syncthreads();
  int64_t g = blockIdx.x;
  if (g >= total) return;
  Acc xa[NS], xb[NS];
  const Tin* __restrict__ p = group_in(g);
  load(p, wave, xa);
  for (;;) {
    const int64_t gn = g + gridDim.x;
    const bool carry = gn < total;
    const Tin* __restrict__ pn = carry ? group_in(gn) : p;   // else a cached reload
    int beta = wave;   // this wave's combinations: wave, wave + kF4Waves, ...
    for (int j = 0; j + 1 < PER; j += 2) {
      load(p, beta + kF4Waves, xb);
      fold(beta, xa);
      beta += kF4Waves;
      load(p, beta + kF4Waves, xa);
      fold(beta, xb);
      beta += kF4Waves;
    }
    load(pn, wave, xb);
    fold(beta, xa);
    lds_barrier();

    const int64_t bs = g / per_outer, c0 = (g % per_outer) * kF4Cols;
    Acc* __restrict__ o = out + bs * NA * L + c0;
    for (int i = tid; i < NA * kF4Cols; i += TH) {
      const Acc v = acc[i];
      acc[i] = Acc(0);
      __builtin_nontemporal_store(v, &o[(int64_t)(i / kF4Cols) * L + (i % kF4Cols)]);
    }
    lds_barrier();
    if (!carry) break;
    g = gn;
    p = pn;
    StaticFor<0, NS>::run([&](auto kc) __attribute__((always_inline)) { xa[decltype(kc)::value] = xb[decltype(kc)::value]; });
  }
}

// ---------------------------------------------------------------------------------
// Row totals: zero fill, per-basis totals (when not supplied), and the final check.

static __global__ void fill_u32_kernel(uint32_t* __restrict__ p, int64_t count, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) p[i] = v;
}

// One block of 256 threads per basis row.
static __global__ __launch_bounds__(256) void row_totals_kernel(const uint16_t* __restrict__ counts,
                                                         int n, uint32_t* __restrict__ nb) {
  const int64_t b = blockIdx.x;
  const int64_t d = (int64_t)1 << n;
  const uint16_t* row = counts + b * d;
  uint32_t s = 0;
  if (n >= 3) {
    // 16-byte loads of 8 counts (rows of 2^n >= 8 counts start 16-byte aligned)
#pragma unroll 4
    for (int64_t i = (int64_t)threadIdx.x * 8; i < d; i += 256 * 8) {
      typedef uint32_t u32x4_v __attribute__((ext_vector_type(4)));
      const u32x4_v v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_v*>(row + i));
      s += (v.x & 0xFFFFu) + (v.x >> 16) + (v.y & 0xFFFFu) + (v.y >> 16) + (v.z & 0xFFFFu) + (v.z >> 16) +
           (v.w & 0xFFFFu) + (v.w >> 16);
    }
  } else {
    for (int64_t i = threadIdx.x; i < d; i += 256) s += row[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  __shared__ uint32_t part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) nb[b] = part[0] + part[1] + part[2] + part[3];
}

// inv[b] = 1 / N_b (0 for an empty basis, which the row check flags), correctly rounded.
static __global__ void reciprocal_kernel(const uint32_t* __restrict__ nb, double* __restrict__ inv, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) inv[i] = nb[i] ? 1.0 / (double)nb[i] : 0.0;
}

// rowpart as written by fold_counts_kernel: [3^n / rows][runs][rows].
// Basis b = grp * rows + j of row group grp.
__device__ __forceinline__ void check_row_gj(const uint32_t* __restrict__ rowpart, int64_t rows, int64_t runs,
                                             const uint32_t* __restrict__ nb, uint64_t shots, int64_t grp, int64_t j,
                                             uint32_t* __restrict__ flags) {
  const int64_t b = grp * rows + j;
  uint64_t tot = 0;
  for (int64_t r = 0; r < runs; ++r) tot += rowpart[(grp * runs + r) * rows + j];
  const uint64_t want = shots ? shots : (uint64_t)nb[b];
  if (tot != want) atomicOr(flags, (uint32_t)FLAG_SHOTS);
  if (!shots && want == 0) atomicOr(flags, (uint32_t)FLAG_EMPTY);
}

__device__ __forceinline__ void check_row(const uint32_t* __restrict__ rowpart, int64_t rows, int64_t runs,
                                          const uint32_t* __restrict__ nb, uint64_t shots, int64_t b,
                                          uint32_t* __restrict__ flags) {
  check_row_gj(rowpart, rows, runs, nb, shots, b / rows, b % rows, flags);
}

static __global__ void check_rows_kernel(const uint32_t* __restrict__ rowpart, int64_t rows, int64_t runs,
                                  const uint32_t* __restrict__ nb, uint64_t shots,
                                  int64_t nbases, uint32_t* __restrict__ flags) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b < nbases) check_row(rowpart, rows, runs, nb, shots, b, flags);
}

// ---------------------------------------------------------------------------------
// Streamed estimation: the counts arrive in slabs of consecutive bases (fixed letters of
// the top h qubits).  Each slab is cut into its 2^h outcome segments (fixed outcome bits
// of the top h qubits); a segment is an instance of n - h qubits whose rows are read with
// the stride of the full rows, and goes through the same passes as any instance, ending
// in unnormalised sums V[s_top][a'].  The top qubits are then folded into the
// coefficient array, which accumulates over the slabs.

// Row totals of a slab: sum the parts every segment's counts pass wrote.
static __global__ void check_rows_seg_kernel(const uint32_t* __restrict__ rowpart, int64_t seg_stride, int nseg,
                                             int64_t rows, int64_t runs, const uint32_t* __restrict__ nb,
                                             uint64_t shots, int64_t nbases, uint32_t* __restrict__ flags) {
  const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (b >= nbases) return;
  const int64_t grp = b / rows, j = b % rows;
  uint64_t tot = 0;
  for (int sg = 0; sg < nseg; ++sg)
    for (int64_t r = 0; r < runs; ++r) tot += rowpart[sg * seg_stride + (grp * runs + r) * rows + j];
  const uint64_t want = shots ? shots : (uint64_t)nb[b];
  if (tot != want) atomicOr(flags, (uint32_t)FLAG_SHOTS);
  if (!shots && want == 0) atomicOr(flags, (uint32_t)FLAG_EMPTY);
}

// Fold of the top H qubits of one slab into the accumulator: for every column a' (the
// letters of the other qubits) and subset m of the top qubits,
//   coef[a_top(m) * ncols + a'] += sum_s (-1)^{|s & m|} V[s][a'],
// a_top(m) carrying letter b_k + 1 at the top qubits in m and I at the others (the
// one-qubit Gamma vectors of Sec. III; the slab fixes the top letters b_k).  Bit / digit
// p of s, m and of the packed letters `atop` belongs to the same qubit (p = 0 lowest).
// Integer sums (uniform shots) stay exact: every value is an integer below 2^53.
template <int H, typename T>
__global__ __launch_bounds__(256) void stream_top_fold_kernel(const T* __restrict__ V, double* __restrict__ coef,
                                                              int64_t ncols, uint32_t atop) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= ncols) return;
  double x[1 << H];
#pragma unroll
  for (int sg = 0; sg < (1 << H); ++sg) x[sg] = acc_to_double(V[(int64_t)sg * ncols + c]);
  wht_regs<H>(x);
#pragma unroll
  for (int m = 0; m < (1 << H); ++m) {
    uint32_t a = 0;
#pragma unroll
    for (int p = 0; p < H; ++p)
      if ((m >> p) & 1) a |= ((atop >> (2 * p)) & 3u) << (2 * p);
    double* dst = coef + (int64_t)a * ncols + c;
    *dst += x[m];
  }
}

// The accumulated sums T_i divided by (X^T X)_ii = 3^{n - w(i)} (and by the shots in
// uniform mode), in place: the coefficients e_i.
static __global__ void stream_finish_kernel(double* __restrict__ coef, int n, uint64_t shots, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const int w = pauli_weight((uint64_t)i);
  coef[i] = shots ? coef[i] / (pow3d(n - w) * (double)shots) : coef[i] / pow3d(n - w);
}

// ---------------------------------------------------------------------------------
// Signed outcome sums of selected rows (verification entry): the low Q bits with the
// same register/lane butterflies as pass 1, the high bits in LDS.  One block per row.
template <int Q>
__global__ __launch_bounds__(256) void signed_sums_kernel(const uint16_t* __restrict__ counts,
                                                          int n, const int64_t* __restrict__ bases,
                                                          int32_t* __restrict__ out,
                                                          uint32_t* __restrict__ flags) {
  using G = Fold1Geom<Q>;
  extern __shared__ int32_t srow[];
  const int64_t d = (int64_t)1 << n;
  const int64_t b = bases[blockIdx.x];
  const bool ok = b >= 0 && b < ipow3(n);
  if (!ok && threadIdx.x == 0) atomicOr(flags, (uint32_t)FLAG_ARG);
  const int tid = threadIdx.x;
  const int grp = tid / G::LPC, lam = tid % G::LPC;
  constexpr int GROUPS = 256 / G::LPC;
  const int64_t nchunks = d >> Q;
  for (int64_t ch = grp; ch < nchunks; ch += GROUPS) {
    int32_t x[G::V];
    if (ok) load_counts<G::V>(counts + b * d + (ch << Q) + lam * G::V, x);
    else
      for (int v = 0; v < G::V; ++v) x[v] = 0;
    wht_regs<G::LB>(x);
    wht_lanes<G::LL, G::V>(x, lam);
    for (int v = 0; v < G::V; ++v) srow[(ch << Q) + lane_walsh<G::LL>(lam) * G::V + v] = x[v];
  }
  __syncthreads();
  for (int bit = Q; bit < n; ++bit) {
    for (int64_t t = tid; t < d / 2; t += 256) {
      const int64_t lo = ((t >> bit) << (bit + 1)) | (t & (((int64_t)1 << bit) - 1));
      const int64_t hi = lo | ((int64_t)1 << bit);
      const int32_t a = srow[lo], c = srow[hi];
      srow[lo] = a + c;
      srow[hi] = a - c;
    }
    __syncthreads();
  }
  for (int64_t t = tid; t < d; t += 256) out[(int64_t)blockIdx.x * d + t] = srow[t];
}

// The same sums with the int8-MFMA form of the counts pass (n >= 6): the 16 columns of
// an MFMA are 16 segments of 64 outcomes of the row, transformed by mfma_wht64; the
// bits above 6 in LDS.  One block (4 waves) per row.
static __global__ __launch_bounds__(256) void signed_sums_mfma_kernel(const uint16_t* __restrict__ counts, int n,
                                                               const int64_t* __restrict__ bases,
                                                               int32_t* __restrict__ out,
                                                               uint32_t* __restrict__ flags) {
  extern __shared__ int32_t srow[];
  const int64_t d = (int64_t)1 << n;
  const int64_t b = bases[blockIdx.x];
  const bool ok = b >= 0 && b < ipow3(n);
  if (!ok && threadIdx.x == 0) atomicOr(flags, (uint32_t)FLAG_ARG);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int col = lane & 15, g = lane >> 4;
  lre_v4i hA[4];
  mfma_h64_operand(col, g, hA);
  const int64_t nseg = d >> 6;
  for (int64_t seg0 = (int64_t)wave * 16; seg0 < nseg; seg0 += 64) {   // uniform per wave
    const int64_t seg = seg0 + col;
    const bool valid = ok && seg < nseg;
    uint32_t w[8];
    if (valid) {
      const uint4* p = reinterpret_cast<const uint4*>(counts + b * d + seg * 64 + 16 * g);
      const uint4 u0 = p[0], u1 = p[1];
      w[0] = u0.x; w[1] = u0.y; w[2] = u0.z; w[3] = u0.w;
      w[4] = u1.x; w[5] = u1.y; w[6] = u1.z; w[7] = u1.w;
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) w[k] = 0;
    }
    int32_t S[4][4];
    mfma_wht64(hA, w, g, S);
    if (seg < nseg) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int r = 0; r < 4; ++r) srow[seg * 64 + 16 * mb + 4 * g + r] = ok ? S[mb][r] : 0;
    }
  }
  __syncthreads();
  for (int bit = 6; bit < n; ++bit) {
    for (int64_t t = tid; t < d / 2; t += 256) {
      const int64_t lo = ((t >> bit) << (bit + 1)) | (t & (((int64_t)1 << bit) - 1));
      const int64_t hi = lo | ((int64_t)1 << bit);
      const int32_t a = srow[lo], c = srow[hi];
      srow[lo] = a + c;
      srow[hi] = a - c;
    }
    __syncthreads();
  }
  for (int64_t t = tid; t < d; t += 256) out[(int64_t)blockIdx.x * d + t] = srow[t];
}

// ---------------------------------------------------------------------------------
// Step (ii).

// (-i)^k applied to (re, im).
__device__ __forceinline__ void mul_neg_i_pow(int k, double& re, double& im) {
  const double r = re, i = im;
  switch (k & 3) {
    case 0: break;
    case 1: re = i; im = -r; break;
    case 2: re = -r; im = -i; break;
    default: re = -i; im = r; break;
  }
}

template <typename OutT>
__device__ __forceinline__ void store_complex(void* base, int64_t idx, double re, double im) {
  if constexpr (sizeof(OutT) == 8) {
    reinterpret_cast<double2*>(base)[idx] = make_double2(re, im);
  } else {
    reinterpret_cast<float2*>(base)[idx] = make_float2((float)re, (float)im);
  }
}

// store_complex with the nontemporal hint (mu is not read again by the library; its
// lines then reach HBM during the kernel instead of being written back from the caches
// during whatever runs next).
template <typename OutT>
__device__ __forceinline__ void store_complex_nt(void* base, int64_t idx, double re, double im) {
  OutT* p = reinterpret_cast<OutT*>(base) + 2 * idx;
  __builtin_nontemporal_store((OutT)re, p);
  __builtin_nontemporal_store((OutT)im, p + 1);
}

// Transform the low J qubits of one 4^J block of coefficients (block = high letters).
// FINAL (J == n): writes mu directly.  Otherwise tmp[a_hi][r_lo][x_lo] (complex128).
template <int J>
struct RhoLowLds {
  static constexpr int D = 1 << J;
  static constexpr int DP = D + 1;  // padded row stride (spreads the rows over LDS banks)
  static constexpr int SIZE = D * DP;  // doubles per plane (re, im)
};

template <int J, bool FINAL, typename OutT, int THREADS>
__device__ __forceinline__ void rho_low_block(const double* __restrict__ coef, void* __restrict__ out,
                                              int n, int64_t a_hi, int tid, double* __restrict__ re,
                                              double* __restrict__ im) {
  constexpr int D = 1 << J;
  constexpr int NN = D * D;
  constexpr int DP = RhoLowLds<J>::DP;   // re, im: [x][z], then [x][r]
  const double* __restrict__ e = coef + a_hi * NN;
  for (int t = tid; t < NN; t += THREADS) {
    int x = 0, z = 0, ny = 0;
#pragma unroll
    for (int p = 0; p < J; ++p) {
      const int dgt = (t >> (2 * p)) & 3;
      x |= (dgt == 1 || dgt == 2) << p;
      z |= (dgt >= 2) << p;
      ny += dgt == 2;
    }
    double vr = e[t], vi = 0.0;
    mul_neg_i_pow(ny, vr, vi);
    re[x * DP + z] = vr;
    im[x * DP + z] = vi;
  }
  __syncthreads();
#pragma unroll 1
  for (int bit = 0; bit < J; ++bit) {
    for (int t = tid; t < NN / 2; t += THREADS) {
      const int x = t / (D / 2), k = t % (D / 2);
      const int lo = ((k >> bit) << (bit + 1)) | (k & ((1 << bit) - 1));
      const int hi = lo | (1 << bit);
      const double a = re[x * DP + lo], b = re[x * DP + hi];
      re[x * DP + lo] = a + b;
      re[x * DP + hi] = a - b;
      const double c = im[x * DP + lo], f = im[x * DP + hi];
      im[x * DP + lo] = c + f;
      im[x * DP + hi] = c - f;
    }
    __syncthreads();
  }
  if constexpr (FINAL) {
    const double scale = ldexp(1.0, -J);  // 2^-n with n == J
    for (int t = tid; t < NN; t += THREADS) {
      const int r = t / D, c = t % D, x = r ^ c;
      store_complex<OutT>(out, t, re[x * DP + r] * scale, im[x * DP + r] * scale);
    }
  } else {
    double2* tmp = static_cast<double2*>(out) + a_hi * NN;
    for (int t = tid; t < NN; t += THREADS) {
      const int r = t / D, x = t % D;
      tmp[t] = make_double2(re[x * DP + r], im[x * DP + r]);
    }
  }
}

template <int J, bool FINAL, typename OutT>
__global__ __launch_bounds__(256) void rho_low_kernel(const double* __restrict__ coef,
                                                      void* __restrict__ out, int n) {
  __shared__ double re[RhoLowLds<J>::SIZE], im[RhoLowLds<J>::SIZE];
  rho_low_block<J, FINAL, OutT, 256>(coef, out, n, blockIdx.x, threadIdx.x, re, im);
}

// Bit p of v moved to bit 2p (6 bits).
__device__ __forceinline__ uint32_t spread6(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int p = 0; p < 6; ++p) r |= ((v >> p) & 1u) << (2 * p);
  return r;
}

// Low transform of one block of 4^6 coefficients (block a_hi).
// The block is staged in LDS with coalesced loads; thread (x, zl) = (t / 4, t % 4)
// gathers its 16 values z = zl + 4k (letter digit x_p ^ 3 z_p: I, X, Y, Z for (x, z)
// bits (0,0), (1,0), (1,1), (0,1)), transforms z bits 2-5 in registers and bits 0-1
// across its lane quad (DPP, exact butterflies), and writes tmp[a_hi][r][x].
// Transform part: blk (LDS) holds the 4096 coefficients of block a_hi; threads 0..255.
__device__ __forceinline__ void rho_low6_from_lds(const double* __restrict__ blk, double2* __restrict__ tmp,
                                                  int64_t a_hi, int t) {
  const uint32_t x = (uint32_t)t >> 2, zl = (uint32_t)t & 3u;
  const uint32_t sx = spread6(x);
  double re[16], im[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const uint32_t z = zl + 4u * (uint32_t)k;
    const uint32_t sz = spread6(z);
    re[k] = blk[sx ^ sz ^ (sz << 1)];
    im[k] = 0.0;
    mul_neg_i_pow(__popc(x & z), re[k], im[k]);
  }
  wht_regs<4>(re);
  wht_regs<4>(im);
  int32_t sg[2] = {(t & 1) ? -1 : 1, (t & 2) ? -1 : 1};
  asm volatile("" : "+v"(sg[0]), "+v"(sg[1]));
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    lane_bfly<kDppQuadXor1, false>(re[k], sg[0]);
    lane_bfly<kDppQuadXor1, false>(im[k], sg[0]);
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    lane_bfly<kDppQuadXor2, false>(re[k], sg[1]);
    lane_bfly<kDppQuadXor2, false>(im[k], sg[1]);
  }
  double2* __restrict__ o = tmp + a_hi * 4096;
#pragma unroll
  for (int k = 0; k < 16; ++k) o[(zl + 4u * (uint32_t)k) * 64u + x] = make_double2(re[k], im[k]);
}

// nz blocks a_hi = a_of(0 .. nz-1) in sequence, the next block's coefficients loaded into
// registers while the current one is transformed.
template <int THREADS, typename AOf>
__device__ __forceinline__ void rho_low6_blocks(const double* __restrict__ coef, double2* __restrict__ tmp,
                                                AOf a_of, int nz, int t, double* __restrict__ blk) {
  constexpr int PER = (4096 + THREADS - 1) / THREADS;
  static_assert(THREADS >= 256, "one thread per (x, z quad)");
  double pre[PER];
  {
    const double* __restrict__ e = coef + a_of(0) * 4096;
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (t + THREADS * i < 4096) pre[i] = e[t + THREADS * i];
  }
  for (int z = 0; z < nz; ++z) {
    lds_barrier();  // the previous block's transform has read blk
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (t + THREADS * i < 4096) blk[t + THREADS * i] = pre[i];
    lds_barrier();
    if (z + 1 < nz) {
      const double* __restrict__ e = coef + a_of(z + 1) * 4096;
#pragma unroll
      for (int i = 0; i < PER; ++i)
        if (t + THREADS * i < 4096) pre[i] = e[t + THREADS * i];
    }
    if (t < 256) rho_low6_from_lds(blk, tmp, a_of(z), t);
  }
}

// Persistent: block b transforms coefficient blocks b, b + gridDim.x, ... < nblk, each
// block's coefficients loaded while the previous one is transformed.
static __global__ __launch_bounds__(256) void rho_low6_kernel(const double* __restrict__ coef, double2* __restrict__ tmp,
                                                              int64_t nblk) {
  __shared__ double blk[4096];
  const int64_t b0 = blockIdx.x, st = gridDim.x;
  if (b0 >= nblk) return;
  const int nz = (int)((nblk - 1 - b0) / st + 1);
  rho_low6_blocks<256>(coef, tmp, [&](int z) { return b0 + (int64_t)z * st; }, nz, threadIdx.x, blk);
}

// Bit p of v moved to bit 2p (B bits).
template <int B>
__device__ __forceinline__ uint32_t spread_bits(uint32_t v) {
  uint32_t r = 0;
#pragma unroll
  for (int p = 0; p < B; ++p) r |= ((v >> p) & 1u) << (2 * p);
  return r;
}

// Letter code of B qubits with x bits x and z bits z (per qubit I, X, Y, Z for (x, z) =
// (0,0), (1,0), (1,1), (0,1)), base-4 digits in the same order as the bits.
template <int B>
__device__ __forceinline__ uint32_t letters_of(uint32_t x, uint32_t z) {
  const uint32_t sz = spread_bits<B>(z);
  return spread_bits<B>(x) ^ sz ^ (sz << 1);
}

// Step (ii) for n = 6 + H <= 10 with no intermediate in device memory.  A unit is a high
// pattern x_hi and 8 consecutive low patterns x_lo = 8 xb + j (unit index 8 x_hi + xb).
// Its inputs are the coefficients of the 2^H blocks a_hi(x_hi, z_hi) whose letters on
// low qubits 3..5 match xb: 2^H x 8 runs of 64 consecutive coefficients (the letters of
// qubits 0..2 free), staged in LDS as V[z_hi][z_lo bits 3..5][letters of qubits 0..2].
// The low transform is real: for each (z_hi, j),
//   T(r_lo) = sum_{z_lo} e (-1)^{floor(|x_lo & z_lo| / 2)} (-1)^{z_lo . r_lo},
// in place (each (j, z_lo) owns one slot; output r_lo goes to the slot of z_lo = r_lo).
// Since (-i)^k = (-1)^{floor(k/2)} (-i)^{k mod 2} and k mod 2 = x_lo . z_lo is a
// character, the complex low transform of e (-i)^{|x_lo & z_lo|} at r_lo is
//   ((T(r_lo) + T(r_lo ^ x_lo)) - i (T(r_lo) - T(r_lo ^ x_lo))) / 2,
// rebuilt per output row from the pair; the high transform over z_hi then runs in
// registers and writes row (r_hi, r_lo), columns (r_hi ^ x_hi, r_lo ^ x_lo): the 8 lanes
// of one r_lo write one 128-byte row segment.  The conjugate entry (row r ^ x) takes the
// same sum and the negated difference and goes through the same butterflies with the
// inputs weighted by a character, so mu is exactly Hermitian.  LDS: 2^H x 512 doubles.
template <int H>
struct RhoTileGeom {
  static constexpr int NZ = 1 << H;
  static constexpr int NV = NZ * 512;  // staged values
};

__device__ __forceinline__ int rho_tile_slot(uint32_t j, uint32_t w6) {
  return (int)(((w6 >> 3) << 6) | letters_of<3>(j, w6 & 7u));
}

// Units [u0, u1) of one instance, in sequence; the next unit's inputs are loaded into
// registers while the current one is transformed.  Every thread of the block calls this.
template <int H, typename OutT, int THREADS>
__device__ __forceinline__ void rho_tiles(const double* __restrict__ coef, void* __restrict__ rho, int64_t u0,
                                          int64_t u1, int t, double* __restrict__ V) {
  using G = RhoTileGeom<H>;
  constexpr int n = 6 + H;
  constexpr int PER = (G::NV + THREADS - 1) / THREADS;
  static_assert(THREADS >= G::NZ * 32, "one lane quad per (z_hi, j) low transform");
  double pre[PER];
  auto load = [&](int64_t u) __attribute__((always_inline)) {
    const uint32_t x_hi = (uint32_t)(u >> 3), xb = (uint32_t)(u & 7);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + THREADS * i;
      if (e < G::NV) {
        const uint32_t z_hi = (uint32_t)e >> 9, zh3 = ((uint32_t)e >> 6) & 7u, l = (uint32_t)e & 63u;
        const int64_t src = ((int64_t)letters_of<H>(x_hi, z_hi) << 12) | (letters_of<3>(xb, zh3) << 6) | l;
        pre[i] = coef[src];
      }
    }
  };
  const double scale = ldexp(1.0, -n - 1);
  if (u0 < u1) load(u0);
  for (int64_t u = u0; u < u1; ++u) {
    lds_barrier();  // the previous unit's high transform has read V
#pragma unroll
    for (int i = 0; i < PER; ++i)
      if (t + THREADS * i < G::NV) V[t + THREADS * i] = pre[i];
    lds_barrier();
    if (u + 1 < u1) load(u + 1);
    const uint32_t x_hi = (uint32_t)(u >> 3), xb = (uint32_t)(u & 7);
    if (t < G::NZ * 32) {  // low transform: lane quad (z_hi, j), lane zl holds z_lo = zl + 4k
      const uint32_t q = (uint32_t)t >> 2, zl = (uint32_t)t & 3u;
      const uint32_t z_hi = q >> 3, j = q & 7u, x_lo = (xb << 3) | j;
      double* __restrict__ Vz = V + z_hi * 512;
      double v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t z = zl + 4u * (uint32_t)k;
        const double a = Vz[rho_tile_slot(j, z)];
        v[k] = (__popc(x_lo & z) & 2) ? -a : a;
      }
      wht_regs<4>(v);
      int32_t sg[2] = {(t & 1) ? -1 : 1, (t & 2) ? -1 : 1};
      asm volatile("" : "+v"(sg[0]), "+v"(sg[1]));
#pragma unroll
      for (int k = 0; k < 16; ++k) lane_bfly<kDppQuadXor1, false>(v[k], sg[0]);
#pragma unroll
      for (int k = 0; k < 16; ++k) lane_bfly<kDppQuadXor2, false>(v[k], sg[1]);
#pragma unroll
      for (int k = 0; k < 16; ++k) Vz[rho_tile_slot(j, zl + 4u * (uint32_t)k)] = v[k];
    }
    lds_barrier();
    for (int w = t; w < 512; w += THREADS) {  // high transform: (r_lo, j), j fastest
      const uint32_t r_lo = (uint32_t)w >> 3, j = (uint32_t)w & 7u;
      const uint32_t rb = r_lo ^ ((xb << 3) | j);
      const int sa = rho_tile_slot(j, r_lo), sb = rho_tile_slot(j, rb);
      double re[G::NZ], im[G::NZ];
#pragma unroll
      for (int z = 0; z < G::NZ; ++z) {
        const double ta = V[z * 512 + sa], tb = V[z * 512 + sb];
        re[z] = ta + tb;
        im[z] = tb - ta;
        mul_neg_i_pow(__popc(x_hi & (uint32_t)z), re[z], im[z]);
      }
      wht_regs<H>(re);
      wht_regs<H>(im);
#pragma unroll
      for (int r_hi = 0; r_hi < G::NZ; ++r_hi) {
        const int64_t row = ((int64_t)r_hi << 6) | r_lo;
        const int64_t col = ((int64_t)(r_hi ^ x_hi) << 6) | rb;
        store_complex<OutT>(rho, (row << n) + col, re[r_hi] * scale, im[r_hi] * scale);
      }
    }
  }
}

// Step (ii) for a single instance with n = 6 + H in [7, 10]: one unit per block.
template <int H, typename OutT>
__global__ __launch_bounds__(512) void rho_tile_kernel(const double* __restrict__ coef, void* __restrict__ rho) {
  __shared__ double V[RhoTileGeom<H>::NV];
  rho_tiles<H, OutT, 512>(coef, rho, blockIdx.x, (int64_t)blockIdx.x + 1, threadIdx.x, V);
}

// Step (ii) for n = 6 + H with no intermediate in device memory, in real arithmetic up
// to the last step (n = 11, 12).  For a fixed pattern x the values
//   g(z) = e_{a(x,z)} (-1)^{floor(|x & z| / 2)}
// are real; with G their n-bit Walsh-Hadamard transform, (-i)^k = (-1)^{floor(k/2)}
// (-i)^{k mod 2} and k mod 2 = x . z (a character of z) give
//   2^n mu[r][r ^ x] = ((G(r) + G(r ^ x)) - i (G(r) - G(r ^ x))) / 2.
// A unit is a high pattern x_hi and XB = 2^JB consecutive low patterns x_lo = XB xb + j
// (unit index (x_hi << (6 - JB)) | xb).  Its inputs, 2^H x 64 x XB coefficients, are
// staged in LDS as V[z_hi][z_lo >> JB][letters of qubits 0..JB-1] (runs of 4^JB
// consecutive coefficients, each z_hi row padded by 16 doubles).  The low transform runs
// per (z_hi, j) in a lane quad (registers and DPP), the high one per slot in two phases
// of at most 3 bits, all in place; every output row then takes one segment of XB
// entries.  Coefficients are read and mu written with the nontemporal hint.  The
// entry at (r ^ x, r) is built from the same two values with the difference negated, so
// mu is exactly Hermitian.
template <int H, int JB>
struct RhoRealGeom {
  static constexpr int XB = 1 << JB, NZ = 1 << H, PZ = 64 * XB, PZP = PZ + 16;
  static constexpr int NV = NZ * PZ, NVP = NZ * PZP;   // values; LDS doubles
  static constexpr int64_t UNITS = (int64_t)NZ << (6 - JB);
};

template <int JB>
__device__ __forceinline__ int rho_real_slot(uint32_t j, uint32_t z_lo) {
  return (int)(((z_lo >> JB) << (2 * JB)) | letters_of<JB>(j, z_lo & ((1u << JB) - 1u)));
}

// Work index -> unit: indices i and i + 8 (consecutive workgroups on one XCD, since
// workgroups go round-robin over the 8 XCDs) get the units of x_lo blocks 2m and 2m + 1,
// which write the two halves of the same rows' 128-byte segments.  A bijection of
// [0, 2^k) for k >= 4.
__device__ __forceinline__ int64_t rho_pair_unit(int64_t i) {
  return ((((i >> 4) << 3) | (i & 7)) << 1) | ((i >> 3) & 1);
}

// Walsh-Hadamard transform over bits [B0, B0 + B) of the row index z of V[z][slot],
// in place, for all PZ slots (rows PZP doubles apart).
template <int H, int B0, int B, int PZ, int PZP, int THREADS>
__device__ __forceinline__ void rho_real_high(double* __restrict__ V, int t) {
  constexpr int NG = (1 << H) >> B;   // values of the other H - B bits
  for (int w = t; w < PZ * NG; w += THREADS) {
    const int s = w % PZ, grp = w / PZ;
    const int base = (grp & ((1 << B0) - 1)) | ((grp >> B0) << (B0 + B));
    double g[1 << B];
#pragma unroll
    for (int k = 0; k < (1 << B); ++k) g[k] = V[(base | (k << B0)) * PZP + s];
    wht_regs<B>(g);
#pragma unroll
    for (int k = 0; k < (1 << B); ++k) V[(base | (k << B0)) * PZP + s] = g[k];
  }
}

// Work indices i0, i0 + istride, ... < UNITS in sequence; the next unit's inputs are
// loaded into registers while the current one is transformed.
template <int H, int JB, typename OutT, int THREADS>
__device__ __forceinline__ void rho_real_units(const double* __restrict__ coef, void* __restrict__ rho, int64_t i0,
                                               int64_t istride, int t, double* __restrict__ V) {
  using G = RhoRealGeom<H, JB>;
  constexpr int n = 6 + H, XB = G::XB, PZ = G::PZ, PZP = G::PZP;
  constexpr uint32_t JM = XB - 1;
  constexpr int PER = (G::NV + THREADS - 1) / THREADS;
  static_assert(THREADS % 4 == 0, "whole lane quads");
  double pre[PER];
  auto load = [&](int64_t u) __attribute__((always_inline)) {
    const uint32_t x_hi = (uint32_t)(u >> (6 - JB)), xb = (uint32_t)u & ((1u << (6 - JB)) - 1u);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = t + THREADS * i;
      if (e < G::NV) {
        const uint32_t z_hi = (uint32_t)e / PZ, w = (uint32_t)e % PZ;
        const uint32_t zh = w >> (2 * JB), l = w & ((1u << (2 * JB)) - 1u);
        pre[i] = __builtin_nontemporal_load(
            &coef[((int64_t)letters_of<H>(x_hi, z_hi) << 12) | (letters_of<6 - JB>(xb, zh) << (2 * JB)) | l]);
      }
    }
  };
  const double scale = ldexp(1.0, -n - 1);
  if (i0 < G::UNITS) load(rho_pair_unit(i0));
  for (int64_t i = i0; i < G::UNITS; i += istride) {
    const int64_t u = rho_pair_unit(i);
    lds_barrier();  // the previous unit's output has read V
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = t + THREADS * k;
      if (e < G::NV) V[(e / PZ) * PZP + e % PZ] = pre[k];
    }
    lds_barrier();
    if (i + istride < G::UNITS) load(rho_pair_unit(i + istride));
    const uint32_t x_hi = (uint32_t)(u >> (6 - JB)), xb = (uint32_t)u & ((1u << (6 - JB)) - 1u);
    // low transform: lane quad (z_hi, j), lane zl holds z_lo = zl + 4k
    for (int q4 = t; q4 < G::NZ * XB * 4; q4 += THREADS) {
      const uint32_t q = (uint32_t)q4 >> 2, zl = (uint32_t)q4 & 3u;
      const uint32_t z_hi = q >> JB, j = q & JM, x_lo = (xb << JB) | j;
      const uint32_t hs = __popc(x_hi & z_hi);
      double* __restrict__ Vz = V + z_hi * PZP;
      double v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t z = zl + 4u * (uint32_t)k;
        const double a = Vz[rho_real_slot<JB>(j, z)];
        v[k] = ((__popc(x_lo & z) + hs) & 2) ? -a : a;
      }
      wht_regs<4>(v);
      int32_t sg[2] = {(q4 & 1) ? -1 : 1, (q4 & 2) ? -1 : 1};
      asm volatile("" : "+v"(sg[0]), "+v"(sg[1]));
#pragma unroll
      for (int k = 0; k < 16; ++k) lane_bfly<kDppQuadXor1, false>(v[k], sg[0]);
#pragma unroll
      for (int k = 0; k < 16; ++k) lane_bfly<kDppQuadXor2, false>(v[k], sg[1]);
#pragma unroll
      for (int k = 0; k < 16; ++k) Vz[rho_real_slot<JB>(j, zl + 4u * (uint32_t)k)] = v[k];
    }
    lds_barrier();
    // high transform: the 2^H values of every slot, z_hi bits 0-2, then the rest
    rho_real_high<H, 0, (H < 3 ? H : 3), PZ, PZP, THREADS>(V, t);
    if constexpr (H > 3) {
      lds_barrier();
      rho_real_high<H, 3, H - 3, PZ, PZP, THREADS>(V, t);
    }
    lds_barrier();
    // output: (r_hi, r_lo, j), j fastest: XB lanes write one row segment
    for (int e = t; e < G::NZ * 64 * XB; e += THREADS) {
      const uint32_t j = (uint32_t)e & JM, r_lo = ((uint32_t)e >> JB) & 63u, r_hi = (uint32_t)e >> (JB + 6);
      const uint32_t rb = r_lo ^ ((xb << JB) | j), rh = r_hi ^ x_hi;
      const double ta = V[r_hi * PZP + rho_real_slot<JB>(j, r_lo)];
      const double tb = V[rh * PZP + rho_real_slot<JB>(j, rb)];
      const int64_t row = ((int64_t)r_hi << 6) | r_lo, col = ((int64_t)rh << 6) | rb;
      store_complex_nt<OutT>(rho, (row << n) + col, (ta + tb) * scale, (tb - ta) * scale);
    }
  }
}

template <int H, int JB, typename OutT>
__global__ __launch_bounds__(512) void rho_real_tile_kernel(const double* __restrict__ coef, void* __restrict__ rho) {
  __shared__ double V[RhoRealGeom<H, JB>::NVP];
  rho_real_units<H, JB, OutT, 512>(coef, rho, blockIdx.x, gridDim.x, threadIdx.x, V);
}

// High transform for H = n - 6 in [7, 9] high qubits, 256 threads.  Block -> (x_hi, r_lo,
// block of XB consecutive x_lo).  z = zA + 16 zB: phase A transforms zA (4 bits) in
// registers per (x_lo, zB) and stores to LDS; phase B transforms zB (H - 4 bits) in
// registers per (x_lo, zA) and writes rows r_hi = zA' + 16 zB' of mu.
template <int H>
struct RhoHigh2Geom {
  static constexpr int D = 64, NH = 1 << H, HB = H - 4, NB = 1 << HB;
  static constexpr int XB = (4096 / NH) < D ? (4096 / NH) : D;  // x_lo values per item
  static constexpr int SP = XB + 1;                              // padded LDS row (one z)
};

// Blocks are persistent (as many as the device holds at once) and walk items
// (x_hi, r_lo, x_lo block) with a stride of the grid; a block loads its next item's
// inputs while it transposes and stores the current one.
template <int H, typename OutT>
__global__ __launch_bounds__(256) void rho_high2_kernel(const double2* __restrict__ tmp, void* __restrict__ rho,
                                                        int n, int64_t items) {
  using G = RhoHigh2Geom<H>;
  constexpr int J = 6, D = G::D, NB = G::NB, HB = G::HB, XB = G::XB, SP = G::SP;
  static_assert(XB * NB <= 256, "phase A takes at most one item per thread");
  __shared__ double sre[G::NH * SP], sim[G::NH * SP];
  const int t = threadIdx.x;
  const bool has_a = t < XB * NB;
  const int xo_a = t % XB, zB_a = t / XB;
  struct Item { int xblk, r_lo, x_hi; };
  auto decode = [&](int64_t it) __attribute__((always_inline)) {
    Item w;
    w.xblk = (int)(it % (D / XB));
    it /= (D / XB);
    w.r_lo = (int)(it % D);
    w.x_hi = (int)(it / D);
    return w;
  };
  // Phase A inputs of item w for this thread: 16 values z = zA + 16 zB_a.
  auto load_a = [&](const Item& w, double (&re)[16], double (&im)[16]) __attribute__((always_inline)) {
    const int x_lo = w.xblk * XB + xo_a;
#pragma unroll
    for (int zA = 0; zA < 16; ++zA) {
      const int z = zA + 16 * zB_a;
      int64_t a_hi = 0;
#pragma unroll
      for (int p = H - 1; p >= 0; --p) {
        const int xb = (w.x_hi >> p) & 1, zb = (z >> p) & 1;
        a_hi = a_hi * 4 + (xb ? (zb ? 2 : 1) : (zb ? 3 : 0));
      }
      const double2 v = tmp[(a_hi * D + w.r_lo) * D + x_lo];
      re[zA] = v.x;
      im[zA] = v.y;
    }
    __builtin_amdgcn_sched_barrier(0);   // issue the loads here, ahead of the current item's work
  };
  const double scale = ldexp(1.0, -n);
  const int64_t dn = (int64_t)1 << n;

  int64_t it = blockIdx.x;
  if (it >= items) return;
  Item w = decode(it);
  double nre[16], nim[16];
  if (has_a) load_a(w, nre, nim);
  for (;;) {
    if (has_a) {
      double re[16], im[16];
#pragma unroll
      for (int zA = 0; zA < 16; ++zA) {
        re[zA] = nre[zA];
        im[zA] = nim[zA];
        mul_neg_i_pow(__popc((unsigned)(w.x_hi & (zA + 16 * zB_a))), re[zA], im[zA]);
      }
      wht_regs<4>(re);
      wht_regs<4>(im);
#pragma unroll
      for (int zA = 0; zA < 16; ++zA) {
        sre[(zA + 16 * zB_a) * SP + xo_a] = re[zA];
        sim[(zA + 16 * zB_a) * SP + xo_a] = im[zA];
      }
    }
    lds_barrier();
    const int64_t nx = it + gridDim.x;
    const Item wn = decode(nx < items ? nx : it);
    if (has_a && nx < items) load_a(wn, nre, nim);
    // phase B: items (xo, zA), xo fastest
    for (int ib = t; ib < XB * 16; ib += 256) {
      const int xo = ib % XB, zA = ib / XB;
      const int x_lo = w.xblk * XB + xo;
      double re[NB], im[NB];
#pragma unroll
      for (int zB = 0; zB < NB; ++zB) {
        re[zB] = sre[(zA + 16 * zB) * SP + xo];
        im[zB] = sim[(zA + 16 * zB) * SP + xo];
      }
      wht_regs<HB>(re);
      wht_regs<HB>(im);
#pragma unroll
      for (int zB = 0; zB < NB; ++zB) {
        const int r_hi = zA + 16 * zB;
        const int64_t row = ((int64_t)r_hi << J) | w.r_lo;
        const int64_t col = ((int64_t)(r_hi ^ w.x_hi) << J) | (w.r_lo ^ x_lo);
        store_complex<OutT>(rho, row * dn + col, re[zB] * scale, im[zB] * scale);
      }
    }
    lds_barrier();
    if (nx >= items) break;
    it = nx;
    w = wn;
  }
}

}  // namespace lre
