/* philox_cpu.c -- host twin of the Philox count workload generator (input
 * generation only).  Same recipe as philox_gen.hip and philox.py:
 *   c[b][s] = (Philox4x32-10(ctr = (s, b lo, b hi, 0), key = (seed lo, seed hi)).x0 * 13) >> 32
 * Philox4x32-10 follows its published definition (Salmon et al., SC'11). */
#include <stdint.h>

static uint32_t philox_x0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                          uint32_t k1) {
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

/* Rows bases[0..nrows) into out[nrows][2^n]; totals into nb (may be NULL).  paired != 0:
 * outcome 2k + 1 gets 12 minus the count of outcome 2k (uniform totals 12 * 2^(n-1)). */
int tomo_philox_rows_mode(int n, uint64_t seed, const int64_t* bases, int64_t nrows, uint16_t* out,
                          uint32_t* nb, int paired) {
  if (n < 1 || n > 20 || !bases || !out) return 1;
  const int64_t d = (int64_t)1 << n;
  const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < nrows; ++j) {
    const uint64_t b = (uint64_t)bases[j];
    uint32_t sum = 0;
    for (int64_t s = 0; s < d; ++s) {
      uint32_t c;
      if (paired && (s & 1)) {
        c = 12u - out[j * d + s - 1];
      } else {
        const uint32_t x = philox_x0((uint32_t)s, (uint32_t)b, (uint32_t)(b >> 32), 0u, k0, k1);
        c = (uint32_t)(((uint64_t)x * 13u) >> 32);
      }
      out[j * d + s] = (uint16_t)c;
      sum += c;
    }
    if (nb) nb[j] = sum;
  }
  return 0;
}

int tomo_philox_rows(int n, uint64_t seed, const int64_t* bases, int64_t nrows, uint16_t* out,
                     uint32_t* nb) {
  return tomo_philox_rows_mode(n, seed, bases, nrows, out, nb, 0);
}
