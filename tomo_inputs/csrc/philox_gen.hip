// philox_gen.hip -- on-device generator of the Philox count workload (input
// generation only; it computes nothing of the estimator).
//
// Philox4x32-10 written from its published definition (Salmon, Moraes, Dror, Shaw,
// SC'11): 10 rounds of two 32x32->64-bit multiplications by fixed odd constants on
// counter words 0 and 2, mixing of the high halves with words 1, 3 and the key, and a
// Weyl increment of the key between rounds.  The numpy twin in tomo_inputs/philox.py
// follows the same recipe; tests compare the two bit for bit.
//
//   c[b][s] = (Philox(ctr = (s, b lo, b hi, 0), key = (seed lo, seed hi)).x0 * 13) >> 32
//   nb[b]   = sum_s c[b][s]
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint32_t philox_x0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
  }
  return c0;
}

__device__ __forceinline__ uint32_t draw(uint64_t s, uint64_t b, uint32_t k0, uint32_t k1) {
  const uint32_t x = philox_x0((uint32_t)s, (uint32_t)b, (uint32_t)(b >> 32), 0u, k0, k1);
  return (uint32_t)(((uint64_t)x * 13u) >> 32);
}

// One block of 256 threads per basis row.  PAIRED: outcome 2k + 1 gets 12 minus the
// count of outcome 2k (every row then sums to 12 * 2^(n-1): a uniform-shot workload).
template <bool PAIRED>
__global__ __launch_bounds__(256) void philox_counts_kernel(int n, uint32_t k0, uint32_t k1,
                                                            int64_t b_begin, uint16_t* __restrict__ counts,
                                                            uint32_t* __restrict__ nb) {
  const int64_t b = b_begin + blockIdx.x;
  const int64_t d = (int64_t)1 << n;
  uint16_t* row = counts + (int64_t)blockIdx.x * d;
  uint32_t sum = 0;
  if (d >= 8) {
    for (int64_t s0 = (int64_t)threadIdx.x * 8; s0 < d; s0 += 256 * 8) {
      uint32_t w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t lo = draw(s0 + 2 * k, b, k0, k1);
        const uint32_t hi = PAIRED ? 12u - lo : draw(s0 + 2 * k + 1, b, k0, k1);
        sum += lo + hi;
        w[k] = lo | (hi << 16);
      }
      *reinterpret_cast<uint4*>(row + s0) = make_uint4(w[0], w[1], w[2], w[3]);
    }
  } else if (threadIdx.x < d) {
    const uint32_t v = (PAIRED && (threadIdx.x & 1)) ? 12u - draw(threadIdx.x - 1, b, k0, k1)
                                                     : draw(threadIdx.x, b, k0, k1);
    row[threadIdx.x] = (uint16_t)v;
    sum = v;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  __shared__ uint32_t part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0 && nb) nb[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

}  // namespace

extern "C" {

// Rows [b_begin, b_begin + b_count) of the n-qubit Philox workload into counts
// ([b_count][2^n] uint16, 16-byte aligned) and their totals into nb ([b_count] uint32,
// may be NULL).  Enqueued on `stream`; returns 0 on success, nonzero otherwise.
static int gen(bool paired, int n, uint64_t seed, int64_t b_begin, int64_t b_count, uint16_t* counts, uint32_t* nb,
               void* stream);

int tomo_gen_philox_counts(int n, uint64_t seed, int64_t b_begin, int64_t b_count,
                           uint16_t* counts, uint32_t* nb, void* stream) {
  return gen(false, n, seed, b_begin, b_count, counts, nb, stream);
}

// The paired variant (outcome 2k + 1 = 12 - outcome 2k; uniform totals 12 * 2^(n-1)).
int tomo_gen_philox_counts_paired(int n, uint64_t seed, int64_t b_begin, int64_t b_count,
                                  uint16_t* counts, uint32_t* nb, void* stream) {
  return gen(true, n, seed, b_begin, b_count, counts, nb, stream);
}

}  // extern "C"

static int gen(bool paired, int n, uint64_t seed, int64_t b_begin, int64_t b_count, uint16_t* counts, uint32_t* nb,
               void* stream) {
  if (n < 1 || n > 16 || b_begin < 0 || b_count < 0 || !counts) return 1;
  if (reinterpret_cast<uintptr_t>(counts) % 16) return 1;
  if (b_count == 0) return 0;
  int64_t done = 0;
  while (done < b_count) {
    const int64_t chunk = (b_count - done) < 0x7fffffffLL ? (b_count - done) : 0x7fffffffLL;
    if (paired)
      hipLaunchKernelGGL(philox_counts_kernel<true>, dim3((unsigned)chunk), dim3(256), 0,
                         static_cast<hipStream_t>(stream), n, (uint32_t)seed, (uint32_t)(seed >> 32),
                         b_begin + done, counts + done * ((int64_t)1 << n), nb ? nb + done : nullptr);
    else
      hipLaunchKernelGGL(philox_counts_kernel<false>, dim3((unsigned)chunk), dim3(256), 0,
                         static_cast<hipStream_t>(stream), n, (uint32_t)seed, (uint32_t)(seed >> 32),
                         b_begin + done, counts + done * ((int64_t)1 << n), nb ? nb + done : nullptr);
    if (hipGetLastError() != hipSuccess) return 2;
    done += chunk;
  }
  return 0;
}


