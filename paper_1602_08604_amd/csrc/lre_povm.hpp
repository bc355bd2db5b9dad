// lre_povm.hpp -- gfx950 kernels for LRE with the reduced measurement set of Sec. VI:
// one informationally complete set of four operators E_j per qubit (the same on every
// qubit), measured as 4^n product outcomes j = sum_k j_k 4^{n-k}.
//
// With G[j][a] = Tr(E_j sigma_a) (4 x 4), every Gamma^(j) is a tensor product of the
// one-qubit rows G[j_k][.] / sqrt 2, so X^T X = 2^-n (x)_k G^T G is a tensor product of
// dense 4 x 4 blocks (not diagonal as for the Pauli bases) and eq. (3) becomes
//   e = 2^{n/2} theta = ((x)_k M) p,   M = 2 (G^T G)^{-1} G^T,   p = c / N.
// The paper counts this as O(8^n) work; applied as n mode products of M it is
// O(n 4^n): every pass below applies M to a few digit positions of the 4^n vector,
// held in registers or LDS, and the last pass divides by N.  Passes work in place on
// the coefficient array (each block writes exactly the elements it read).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lre_kernels.hpp"

namespace lre {

// M from G (row-major 4 x 4) by Gauss-Jordan elimination with partial pivoting on
// G^T G in binary64; a (nearly) singular G^T G raises FLAG_ARG and leaves M = 0.
// Also clears the 64-bit total N that the first pass accumulates.
static __global__ void povm_setup_kernel(const double* __restrict__ G, double* __restrict__ M,
                                         unsigned long long* __restrict__ total, uint32_t* __restrict__ flags) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  *total = 0ull;
  double g[4][4], a[4][8];
  for (int j = 0; j < 4; ++j)
    for (int c = 0; c < 4; ++c) g[j][c] = G[4 * j + c];
  double scale = 0.0;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int j = 0; j < 4; ++j) s += g[j][r] * g[j][c];
      a[r][c] = s;
      a[r][c + 4] = r == c ? 1.0 : 0.0;
      scale = fmax(scale, fabs(s));
    }
  bool ok = scale > 0.0;
  for (int c = 0; c < 4 && ok; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
    if (!(fabs(a[piv][c]) > 1e-12 * scale)) { ok = false; break; }
    if (piv != c)
      for (int k = 0; k < 8; ++k) { const double t = a[c][k]; a[c][k] = a[piv][k]; a[piv][k] = t; }
    const double d = a[c][c];
    for (int k = 0; k < 8; ++k) a[c][k] /= d;
    for (int r = 0; r < 4; ++r)
      if (r != c) {
        const double f = a[r][c];
        for (int k = 0; k < 8; ++k) a[r][k] -= f * a[c][k];
      }
  }
  for (int r = 0; r < 4; ++r)
    for (int j = 0; j < 4; ++j) {
      double s = 0.0;
      if (ok)
        for (int c = 0; c < 4; ++c) s += a[r][c + 4] * g[j][c];   // (G^T G)^{-1} G^T
      M[4 * r + j] = 2.0 * s;
    }
  if (!ok) atomicOr(flags, (uint32_t)FLAG_ARG);
}

// Empty data (N = 0) is an error, as an empty basis is for the Pauli measurements
// (checked after the first pass has summed the counts).
static __global__ void povm_check_kernel(const unsigned long long* __restrict__ total, uint32_t* __restrict__ flags) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && *total == 0ull) atomicOr(flags, (uint32_t)FLAG_EMPTY);
}

// y <- M y on one digit: 4 values.
__device__ __forceinline__ void povm_apply1(const double (&m)[16], double* y, int stride) {
  const double y0 = y[0], y1 = y[stride], y2 = y[2 * stride], y3 = y[3 * stride];
#pragma unroll
  for (int r = 0; r < 4; ++r)
    y[r * stride] = m[4 * r] * y0 + m[4 * r + 1] * y1 + m[4 * r + 2] * y2 + m[4 * r + 3] * y3;
}

// y <- (M (x) ... (x) M) y on the F digits of a register block of 4^F values.
template <int F>
__device__ __forceinline__ void povm_apply_regs(const double (&m)[16], double* y) {
#pragma unroll
  for (int d = 0; d < F; ++d) {
    const int st = 1 << (2 * d);
#pragma unroll
    for (int base = 0; base < (1 << (2 * F)); ++base) {
      if ((base >> (2 * d)) & 3) continue;
      povm_apply1(m, y + base, st);
    }
  }
}

__device__ __forceinline__ void povm_load_m(const double* __restrict__ M, double (&m)[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) m[k] = M[k];
}

// LDS index of tile element i: one pad slot every 16, so that the 16-value groups of
// the first stage (16 consecutive elements per thread) fall on different banks.
__device__ __forceinline__ int povm_pad(int i) { return i + (i >> 4); }

// First pass: a tile of 4^J consecutive counts (the J lowest digits) in LDS, the J
// digits transformed two at a time in registers (one at a time for an odd J), then
// written to coef.  The tile's counts are summed on the way in: with J < n the block
// adds its sum to N (the last pass divides); with J = n (one block, the only pass) its
// sum is N and the block divides.
template <int J, bool FINAL>
__global__ __launch_bounds__(256) void povm_low_kernel(const uint16_t* __restrict__ counts, double* __restrict__ coef,
                                                       const double* __restrict__ M,
                                                       unsigned long long* __restrict__ total,
                                                       uint32_t* __restrict__ flags) {
  constexpr int T = 1 << (2 * J);
  __shared__ double tile[T + T / 16 + 1];
  __shared__ uint64_t part[4];
  double m[16];
  povm_load_m(M, m);
  const int64_t base = (int64_t)blockIdx.x * T;
  uint64_t sum = 0;
  if constexpr (T >= 8 * 256) {
    // 16-byte loads: 8 counts per thread and step
    for (int i = threadIdx.x * 8; i < T; i += 256 * 8) {
      const uint4 u = *reinterpret_cast<const uint4*>(counts + base + i);
      const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t lo = w[k] & 0xFFFFu, hi = w[k] >> 16;
        tile[povm_pad(i + 2 * k)] = (double)lo;
        tile[povm_pad(i + 2 * k + 1)] = (double)hi;
        sum += lo + hi;
      }
    }
  } else {
    for (int i = threadIdx.x; i < T; i += 256) {
      const uint32_t c = counts[base + i];
      tile[povm_pad(i)] = (double)c;
      sum += c;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  const uint64_t bsum = part[0] + part[1] + part[2] + part[3];
  if (!FINAL && threadIdx.x == 0) atomicAdd(total, (unsigned long long)bsum);
  if (FINAL && threadIdx.x == 0 && bsum == 0) atomicOr(flags, (uint32_t)FLAG_EMPTY);
#pragma unroll
  for (int d = 0; d < J; d += 2) {
    const int nd = (J - d) >= 2 ? 2 : 1;          // digits in this stage
    const int G = T >> (2 * nd);                  // groups of 4^nd values
    for (int g = threadIdx.x; g < G; g += 256) {
      // element index: digits d, d+1 vary; the others come from g
      const int lo = g & ((1 << (2 * d)) - 1);
      const int hi = g >> (2 * d);
      const int i0 = (hi << (2 * (d + nd))) | lo;
      double y[16];
      const int st = 1 << (2 * d);
      if (nd == 2) {
#pragma unroll
        for (int k = 0; k < 16; ++k) y[k] = tile[povm_pad(i0 + (k & 3) * st + (k >> 2) * 4 * st)];
        povm_apply_regs<2>(m, y);
#pragma unroll
        for (int k = 0; k < 16; ++k) tile[povm_pad(i0 + (k & 3) * st + (k >> 2) * 4 * st)] = y[k];
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) y[k] = tile[povm_pad(i0 + k * st)];
        povm_apply1(m, y, 1);
#pragma unroll
        for (int k = 0; k < 4; ++k) tile[povm_pad(i0 + k * st)] = y[k];
      }
    }
    __syncthreads();
  }
  const double N = (double)bsum;
  for (int i = threadIdx.x; i < T; i += 256) coef[base + i] = FINAL ? tile[povm_pad(i)] / N : tile[povm_pad(i)];
}

// Four digits lo .. lo + 3 (lo >= 3) of the vector, in place: a block holds 32
// consecutive low indices (columns) x the 256 values of the four digits in LDS (64 KiB,
// two blocks per compute unit), transforms them two digits at a time in registers;
// FINAL divides by N.
constexpr int kPovmCols = 32;
constexpr int kPovmHighThreads = 512;

template <bool FINAL>
__global__ __launch_bounds__(kPovmHighThreads) void povm_high4_kernel(double* __restrict__ coef, int n, int lo,
                                                                      const double* __restrict__ M,
                                                                      const unsigned long long* __restrict__ total) {
  constexpr int TH = kPovmHighThreads, RPP = TH / kPovmCols;   // rows of 256 loaded per pass
  __shared__ double blk[256 * kPovmCols];
  double m[16];
  povm_load_m(M, m);
  const int64_t L = (int64_t)1 << (2 * lo);            // low indices
  const int64_t colgroups = L / kPovmCols;
  const int64_t hi = blockIdx.x / colgroups;
  const int64_t c0 = (blockIdx.x % colgroups) * kPovmCols;
  double* __restrict__ base = coef + hi * (L << 8) + c0;
  const int col = threadIdx.x % kPovmCols, r0 = threadIdx.x / kPovmCols;
  double v[256 / RPP];
#pragma unroll
  for (int k = 0; k < 256 / RPP; ++k) v[k] = base[(int64_t)(r0 + RPP * k) * L + col];
#pragma unroll
  for (int k = 0; k < 256 / RPP; ++k) blk[(r0 + RPP * k) * kPovmCols + col] = v[k];
  __syncthreads();
#pragma unroll
  for (int stage = 0; stage < 2; ++stage) {
    // units: (column, the other two digits) = 32 x 16, one per thread
    for (int u = threadIdx.x; u < kPovmCols * 16; u += TH) {
      const int c = u % kPovmCols, other = u / kPovmCols;
      double y[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int d = stage == 0 ? (other << 4) | k : (k << 4) | other;
        y[k] = blk[d * kPovmCols + c];
      }
      povm_apply_regs<2>(m, y);
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int d = stage == 0 ? (other << 4) | k : (k << 4) | other;
        blk[d * kPovmCols + c] = y[k];
      }
    }
    __syncthreads();
  }
  const double N = FINAL ? (double)*total : 1.0;
#pragma unroll
  for (int k = 0; k < 256 / RPP; ++k) {
    const int d = r0 + RPP * k;
    base[(int64_t)d * L + col] = FINAL ? blk[d * kPovmCols + col] / N : blk[d * kPovmCols + col];
  }
}

// F <= 3 digits lo .. lo + F - 1 in registers, one thread per column (every other
// digit), in place; FINAL divides by N.
template <int F, bool FINAL>
__global__ __launch_bounds__(256) void povm_reg_kernel(double* __restrict__ coef, int n, int lo,
                                                       const double* __restrict__ M,
                                                       const unsigned long long* __restrict__ total) {
  const int64_t L = (int64_t)1 << (2 * lo);
  const int64_t cols = ((int64_t)1 << (2 * (n - F)));
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= cols) return;
  double m[16];
  povm_load_m(M, m);
  const int64_t low = t & (L - 1), hi = t >> (2 * lo);
  double* __restrict__ p = coef + hi * (L << (2 * F)) + low;
  double y[1 << (2 * F)];
#pragma unroll
  for (int k = 0; k < (1 << (2 * F)); ++k) y[k] = p[(int64_t)k * L];
  povm_apply_regs<F>(m, y);
  const double N = FINAL ? (double)*total : 1.0;
#pragma unroll
  for (int k = 0; k < (1 << (2 * F)); ++k) p[(int64_t)k * L] = FINAL ? y[k] / N : y[k];
}

}  // namespace lre
