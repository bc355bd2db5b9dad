/*
 * lre_oracle.c -- plain CPU oracle for linear regression estimation (LRE) of an
 * n-qubit state from local Pauli measurement counts.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py load this library.  It shares no code, header,
 * table or constant with the HIP library: every quantity below is derived here
 * from the definitions in the paper (Hou et al., "Full reconstruction of a
 * 14-qubit state within four hours", arXiv:1602.08604).
 *
 * What is computed, in the paper's order:
 *   Sec. III, eq. (5): representation basis Omega_i = 2^{-n/2} (x)_k sigma_{i_k},
 *                      i = sum_k i_k 4^{n-k}, sigma_0..3 = I, X, Y, Z.
 *   Sec. II,  eq. (2): vector form of a projector, gamma_i = Tr(P Omega_i).
 *   Sec. III (one-qubit worked case): the 6 one-qubit Gamma vectors and
 *                      X^T X = diag{3,1,1,1}; the n-qubit Gamma and X^T X are
 *                      tensor products of these.
 *   Sec. II,  eq. (3): Theta_LS = (X^T X)^{-1} sum_j p_j Gamma^(j).
 *   Sec. II,  eq. (4): mu = sum_i theta_i Omega_i.
 * Only the terms that are not identically zero are visited (Sec. III: 2^n of the
 * 4^n entries of each Gamma, 2^n nonzero entries per Omega_i), which is the
 * paper's own O(12^n) / O(8^n) evaluation, not a fast transform.
 *
 * Readings where the paper is silent:
 *   - basis index b = sum_k b_k 3^{n-k}, b_k in {0:X, 1:Y, 2:Z}, qubit 1 most
 *     significant (mirrors the Pauli index of eq. 5);
 *   - outcome index s = sum_k s_k 2^{n-k}; s_k = 0 is the +1 eigenvector;
 *   - p_j is the frequency within its basis, c[b][s] / N_b (Sec. V: each basis
 *     is one complete POVM measured at once); this is what makes Tr mu = 1;
 *   - the returned coefficient is the Pauli expectation e_i = 2^{n/2} theta_i,
 *     so e_0 = 1 for every valid input;
 *   - counts are integers, so every signed count sum is exact (int64) and with
 *     uniform shots e_i is one correctly rounded IEEE division; with per-basis
 *     totals the frequency-weighted sums are accumulated in long double.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_N 16

enum {
  ORACLE_OK = 0,
  ORACLE_E_ARG = 1,
  ORACLE_E_SHOTS = 2,       /* a basis row does not sum to the declared shots */
  ORACLE_E_EMPTY_BASIS = 3, /* a basis has no counts, so p = c / N_b is undefined */
  ORACLE_E_TABLE = 4        /* the one-qubit tables did not come out integral */
};

/* ---- one-qubit objects, built from the matrices printed in Sec. III ---- */

static double complex sigma[4][2][2];
/* g[a][b][s] = Tr(P_{b,s} sigma_a), an integer in {0, +1, -1}. */
static int g1[4][3][2];
/* (X^T X) for one qubit, diag{3,1,1,1} (Sec. III), stored in full. */
static double xtx1[4][4];
static int tables_ready = 0;
static int tables_status = ORACLE_OK;

/* Operation counters: one tick per (projector, coefficient) term of eq. (3) and
 * per (coefficient, matrix entry) term of eq. (4) that the oracle visits. */
static uint64_t ops_step1 = 0, ops_step2 = 0;

static void build_tables(void) {
  memset(sigma, 0, sizeof sigma);
  sigma[0][0][0] = 1; sigma[0][1][1] = 1;                 /* I */
  sigma[1][0][1] = 1; sigma[1][1][0] = 1;                 /* X */
  sigma[2][0][1] = -I; sigma[2][1][0] = I;                /* Y */
  sigma[3][0][0] = 1; sigma[3][1][1] = -1;                /* Z */

  /* Projector onto the eigenvector of sigma_{b+1} with eigenvalue (-1)^s:
   * P = (I + (-1)^s sigma_{b+1}) / 2.  All entries are exact in binary64. */
  double gam[3][2][4];
  for (int b = 0; b < 3; ++b)
    for (int s = 0; s < 2; ++s) {
      double complex P[2][2];
      double sgn = s ? -1.0 : 1.0;
      for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c)
          P[r][c] = 0.5 * (sigma[0][r][c] + sgn * sigma[b + 1][r][c]);
      for (int a = 0; a < 4; ++a) {
        /* Tr(P sigma_a) */
        double complex tr = 0;
        for (int r = 0; r < 2; ++r)
          for (int c = 0; c < 2; ++c) tr += P[r][c] * sigma[a][c][r];
        double re = creal(tr);
        if (fabs(cimag(tr)) != 0.0 || re != nearbyint(re)) tables_status = ORACLE_E_TABLE;
        g1[a][b][s] = (int)nearbyint(re);
        gam[b][s][a] = re / sqrt(2.0); /* one-qubit gamma of eq. (2) */
      }
    }
  /* X^T X = sum_j Gamma_j Gamma_j^T over the 6 one-qubit projectors, computed as
   * (1/2) sum g g so that it is exact. */
  for (int a = 0; a < 4; ++a)
    for (int a2 = 0; a2 < 4; ++a2) {
      int acc = 0;
      for (int b = 0; b < 3; ++b)
        for (int s = 0; s < 2; ++s) acc += g1[a][b][s] * g1[a2][b][s];
      xtx1[a][a2] = 0.5 * acc;
    }
  /* The tensor-product shortcut below needs X^T X diagonal (Sec. III). */
  for (int a = 0; a < 4; ++a)
    for (int a2 = 0; a2 < 4; ++a2)
      if (a != a2 && xtx1[a][a2] != 0.0) tables_status = ORACLE_E_TABLE;
  (void)gam;
  tables_ready = 1;
}

static int ensure_tables(void) {
  if (!tables_ready) {
#pragma omp critical(oracle_tables)
    {
      if (!tables_ready) build_tables();
    }
  }
  return tables_status;
}

/* Exported for the pin tests: the 6 one-qubit Gamma vectors (rows ordered
 * X+, X-, Y+, Y-, Z+, Z-) and the one-qubit X^T X. */
int oracle_one_qubit_tables(double gamma_out[6][4], double xtx_out[4][4]) {
  int st = ensure_tables();
  for (int b = 0; b < 3; ++b)
    for (int s = 0; s < 2; ++s)
      for (int a = 0; a < 4; ++a) gamma_out[2 * b + s][a] = g1[a][b][s] / sqrt(2.0);
  memcpy(xtx_out, xtx1, sizeof xtx1);
  return st;
}

/* ---- index helpers (pure digit arithmetic of the conventions) ---- */

static int64_t ipow(int64_t base, int e) {
  int64_t r = 1;
  while (e-- > 0) r *= base;
  return r;
}

static void pauli_digits(int n, int64_t i, int a[ORACLE_MAX_N]) {
  for (int k = n - 1; k >= 0; --k) { a[k] = (int)(i % 4); i /= 4; }
}

/* Diagonal entry (X^T X)_ii = prod_k xtx1[a_k][a_k]  (tensor product, Sec. III). */
static double xtx_diag(int n, const int a[ORACLE_MAX_N]) {
  double d = 1.0;
  for (int k = 0; k < n; ++k) d *= xtx1[a[k]][a[k]];
  return d;
}

/* Bases b whose Gamma has a nonzero entry at coefficient i: for each qubit the
 * letters b_k with g1[a_k][b_k][.] != 0.  Returned as a list per qubit. */
static int allowed_letters(int a_k, int out[3]) {
  int m = 0;
  for (int b = 0; b < 3; ++b)
    if (g1[a_k][b][0] != 0 || g1[a_k][b][1] != 0) out[m++] = b;
  return m;
}

/* Signed count sum of one basis row against coefficient i:
 *   sum_s c[b][s] * prod_k g1[a_k][b_k][s_k]
 * i.e. 2^{n/2} * sum_{s} c[b][s] * gamma_i^{(b,s)}.  Exact in int64. */
static int64_t basis_term(int n, const uint16_t* row, const int a[ORACLE_MAX_N],
                          const int bd[ORACLE_MAX_N]) {
  int64_t S = 0, d = (int64_t)1 << n;
  for (int64_t s = 0; s < d; ++s) {
    int prod = 1;
    for (int k = 0; k < n; ++k) {
      int sk = (int)((s >> (n - 1 - k)) & 1);
      prod *= g1[a[k]][bd[k]][sk];
    }
    S += (int64_t)row[s] * prod;
  }
  return S;
}

/* Iterate over the bases compatible with a[]: odometer over the allowed letters. */
typedef struct {
  int n, nl[ORACLE_MAX_N], lt[ORACLE_MAX_N][3], pos[ORACLE_MAX_N], bd[ORACLE_MAX_N];
  int64_t b;
  int done;
} basis_iter;

static void biter_init(basis_iter* it, int n, const int a[ORACLE_MAX_N]) {
  it->n = n;
  it->done = 0;
  for (int k = 0; k < n; ++k) {
    it->nl[k] = allowed_letters(a[k], it->lt[k]);
    it->pos[k] = 0;
    if (it->nl[k] == 0) it->done = 1;
  }
  it->b = 0;
  for (int k = 0; k < n; ++k) { it->bd[k] = it->lt[k][0]; it->b = it->b * 3 + it->bd[k]; }
}

static void biter_next(basis_iter* it) {
  int k = it->n - 1;
  while (k >= 0) {
    if (++it->pos[k] < it->nl[k]) break;
    it->pos[k] = 0;
    --k;
  }
  if (k < 0) { it->done = 1; return; }
  it->b = 0;
  for (int q = 0; q < it->n; ++q) { it->bd[q] = it->lt[q][it->pos[q]]; it->b = it->b * 3 + it->bd[q]; }
}

static int row_sum_check(int n, const uint16_t* counts, uint64_t shots, const uint32_t* nb) {
  int64_t B = ipow(3, n), d = (int64_t)1 << n;
  int bad = 0;
#pragma omp parallel for reduction(| : bad) schedule(static)
  for (int64_t b = 0; b < B; ++b) {
    uint64_t sum = 0;
    for (int64_t s = 0; s < d; ++s) sum += counts[b * d + s];
    uint64_t want = shots ? shots : (nb ? nb[b] : sum);
    if (sum != want) bad |= 1;
    if (want == 0) bad |= 2;
  }
  if (bad & 2) return ORACLE_E_EMPTY_BASIS;
  if (bad & 1) return ORACLE_E_SHOTS;
  return ORACLE_OK;
}

/* ---- step (i): eq. (3), one coefficient at a time ---- */

/* T_i = 2^{n/2} * sum_j c_j gamma_i^(j)  (integer; the numerator of eq. 3 with
 * uniform shots).  counts: [3^n][2^n] row-major. */
int oracle_pauli_sums(int n, const uint16_t* counts, const int64_t* idx, int64_t nidx,
                      int64_t* T_out) {
  if (n < 1 || n > ORACLE_MAX_N || !counts || !T_out) return ORACLE_E_ARG;
  int st = ensure_tables();
  if (st) return st;
  int64_t d = (int64_t)1 << n, D2 = ipow(4, n);
  int64_t cnt = idx ? nidx : D2;
  uint64_t ops = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : ops)
  for (int64_t t = 0; t < cnt; ++t) {
    int64_t i = idx ? idx[t] : t;
    int a[ORACLE_MAX_N];
    pauli_digits(n, i, a);
    int64_t T = 0;
    basis_iter it;
    for (biter_init(&it, n, a); !it.done; biter_next(&it)) {
      T += basis_term(n, counts + it.b * d, a, it.bd);
      ops += (uint64_t)d;
    }
    T_out[t] = T;
  }
#pragma omp atomic
  ops_step1 += ops;
  return ORACLE_OK;
}

/* Per-basis signed sums used as a cross-check of an intermediate: for basis b and
 * coefficient i (which must be compatible with b), sum_s c[b][s] prod_k g. */
int oracle_basis_sums(int n, const uint16_t* counts, const int64_t* bases, const int64_t* coefs,
                      int64_t npairs, int64_t* out) {
  if (n < 1 || n > ORACLE_MAX_N || !counts || !bases || !coefs || !out) return ORACLE_E_ARG;
  int st = ensure_tables();
  if (st) return st;
  int64_t d = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < npairs; ++t) {
    int a[ORACLE_MAX_N], bd[ORACLE_MAX_N];
    pauli_digits(n, coefs[t], a);
    int64_t b = bases[t];
    for (int k = n - 1; k >= 0; --k) { bd[k] = (int)(b % 3); b /= 3; }
    out[t] = basis_term(n, counts + bases[t] * d, a, bd);
  }
  return ORACLE_OK;
}

/* e_i for a list of coefficients (idx == NULL: all 4^n).
 *   shots > 0 : every basis has exactly `shots` counts (checked);
 *               e_i = T_i / ((X^T X)_ii * shots), one IEEE division.
 *   shots == 0: N_b = nb[b] (checked against the row sum) or the row sum when
 *               nb == NULL; e_i = (X^T X)_ii^{-1} sum_b (1/N_b) sum_s c gamma.   */
int oracle_coefs(int n, const uint16_t* counts, uint64_t shots, const uint32_t* nb,
                 const int64_t* idx, int64_t nidx, double* e_out) {
  if (n < 1 || n > ORACLE_MAX_N || !counts || !e_out) return ORACLE_E_ARG;
  int st = ensure_tables();
  if (st) return st;
  st = row_sum_check(n, counts, shots, nb);
  if (st) return st;
  int64_t d = (int64_t)1 << n, D2 = ipow(4, n);
  int64_t cnt = idx ? nidx : D2;
  uint64_t ops = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : ops)
  for (int64_t t = 0; t < cnt; ++t) {
    int64_t i = idx ? idx[t] : t;
    int a[ORACLE_MAX_N];
    pauli_digits(n, i, a);
    double xtx = xtx_diag(n, a);
    basis_iter it;
    if (shots) {
      int64_t T = 0;
      for (biter_init(&it, n, a); !it.done; biter_next(&it)) {
        T += basis_term(n, counts + it.b * d, a, it.bd);
        ops += (uint64_t)d;
      }
      e_out[t] = (double)T / (xtx * (double)shots);
    } else {
      long double acc = 0.0L;
      for (biter_init(&it, n, a); !it.done; biter_next(&it)) {
        const uint16_t* row = counts + it.b * d;
        uint64_t Nb = 0;
        if (nb) Nb = nb[it.b];
        else
          for (int64_t s = 0; s < d; ++s) Nb += row[s];
        int64_t S = basis_term(n, row, a, it.bd);
        acc += (long double)S / (long double)Nb;
        ops += (uint64_t)d;
      }
      e_out[t] = (double)(acc / (long double)xtx);
    }
  }
#pragma omp atomic
  ops_step1 += ops;
  return ORACLE_OK;
}

/* e_i from basis rows supplied explicitly (used where the whole count tensor does
 * not fit in host memory): rows[j] is the row of the j-th basis compatible with
 * coefficient i, in increasing b order, and nb[j] its total.  Same arithmetic as
 * the per-basis branch of oracle_coefs. */
int oracle_coef_from_rows(int n, int64_t i, const uint16_t* rows, const uint32_t* nb,
                          int64_t nrows, double* e_out) {
  if (n < 1 || n > ORACLE_MAX_N || !rows || !nb || !e_out) return ORACLE_E_ARG;
  int st = ensure_tables();
  if (st) return st;
  int a[ORACLE_MAX_N];
  pauli_digits(n, i, a);
  int64_t d = (int64_t)1 << n;
  basis_iter it;
  long double acc = 0.0L;
  int64_t j = 0;
  for (biter_init(&it, n, a); !it.done; biter_next(&it), ++j) {
    if (j >= nrows) return ORACLE_E_ARG;
    if (nb[j] == 0) return ORACLE_E_EMPTY_BASIS;
    uint64_t sum = 0;
    for (int64_t s = 0; s < d; ++s) sum += rows[j * d + s];
    if (sum != nb[j]) return ORACLE_E_SHOTS;
    acc += (long double)basis_term(n, rows + j * d, a, it.bd) / (long double)nb[j];
  }
  if (j != nrows) return ORACLE_E_ARG;
  *e_out = (double)(acc / (long double)xtx_diag(n, a));
  return ORACLE_OK;
}

/* Streaming form of the per-basis branch of eq. (3), for count tensors too large to
 * hold (the 14-qubit workload): the caller regenerates basis rows in chunks and names
 * the (row, coefficient) pairs to evaluate; pairs must be compatible (basis b ~ i), which
 * the caller takes from oracle_compatible_bases.  For pair p, with j = pair_row[p]:
 *   acc[pair_slot[p]] += (sum_s rows[j][s] prod_k g(a_k, b_k, s_k)) / nb[j]
 * in long double, pairs added in the order given (the per-pair terms are computed in
 * parallel, the additions run serially, so the result does not depend on threads).
 * Each row's total is checked against nb[j].  After every compatible basis of i has
 * been visited, e_i = acc / (X^T X)_ii (oracle_coef_from_acc). */
int oracle_accumulate_pairs(int n, const uint16_t* rows, const int64_t* bases, const uint32_t* nb,
                            int64_t nrows, const int64_t* pair_row, const int64_t* pair_coef,
                            const int64_t* pair_slot, int64_t npairs, long double* acc) {
  if (n < 1 || n > ORACLE_MAX_N || !rows || !bases || !nb || !acc || (npairs && (!pair_row || !pair_coef || !pair_slot)))
    return ORACLE_E_ARG;
  int st = ensure_tables();
  if (st) return st;
  int64_t d = (int64_t)1 << n;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t j = 0; j < nrows; ++j) {
    uint64_t sum = 0;
    for (int64_t s = 0; s < d; ++s) sum += rows[j * d + s];
    if (nb[j] == 0) bad |= 2;
    else if (sum != nb[j]) bad |= 1;
  }
  if (bad & 2) return ORACLE_E_EMPTY_BASIS;
  if (bad & 1) return ORACLE_E_SHOTS;
  long double* term = (long double*)malloc(sizeof(long double) * (size_t)(npairs > 0 ? npairs : 1));
  if (!term) return ORACLE_E_ARG;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
  for (int64_t p = 0; p < npairs; ++p) {
    int64_t j = pair_row[p];
    if (j < 0 || j >= nrows) { bad |= 1; term[p] = 0.0L; continue; }
    int a[ORACLE_MAX_N], bd[ORACLE_MAX_N];
    pauli_digits(n, pair_coef[p], a);
    int64_t b = bases[j];
    for (int k = n - 1; k >= 0; --k) { bd[k] = (int)(b % 3); b /= 3; }
    term[p] = (long double)basis_term(n, rows + j * d, a, bd) / (long double)nb[j];
  }
  if (bad) { free(term); return ORACLE_E_ARG; }
  for (int64_t p = 0; p < npairs; ++p) acc[pair_slot[p]] += term[p];
  free(term);
  return ORACLE_OK;
}

/* e_i from its completed sum over compatible bases (oracle_accumulate_pairs):
 * (X^T X)^{-1}_ii * acc, the last step of eq. (3). */
int oracle_coef_from_acc(int n, const int64_t* coefs, const long double* acc, int64_t count, double* e_out) {
  if (n < 1 || n > ORACLE_MAX_N || !coefs || !acc || !e_out) return ORACLE_E_ARG;
  int st = ensure_tables();
  if (st) return st;
  for (int64_t t = 0; t < count; ++t) {
    int a[ORACLE_MAX_N];
    pauli_digits(n, coefs[t], a);
    e_out[t] = (double)(acc[t] / (long double)xtx_diag(n, a));
  }
  return ORACLE_OK;
}

/* Number of bases compatible with coefficient i, and their indices in increasing
 * order (out may be NULL to only count). */
int64_t oracle_compatible_bases(int n, int64_t i, int64_t* out) {
  if (ensure_tables()) return -1;
  int a[ORACLE_MAX_N];
  pauli_digits(n, i, a);
  basis_iter it;
  int64_t m = 0;
  for (biter_init(&it, n, a); !it.done; biter_next(&it)) {
    if (out) out[m] = it.b;
    ++m;
  }
  return m;
}

/* Eq. (3) with exact frequencies p[b][s] (double) instead of counts. */
int oracle_coefs_freq(int n, const double* freq, const int64_t* idx, int64_t nidx,
                      double* e_out) {
  if (n < 1 || n > ORACLE_MAX_N || !freq || !e_out) return ORACLE_E_ARG;
  int st = ensure_tables();
  if (st) return st;
  int64_t d = (int64_t)1 << n, D2 = ipow(4, n);
  int64_t cnt = idx ? nidx : D2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < cnt; ++t) {
    int64_t i = idx ? idx[t] : t;
    int a[ORACLE_MAX_N];
    pauli_digits(n, i, a);
    long double acc = 0.0L;
    basis_iter it;
    for (biter_init(&it, n, a); !it.done; biter_next(&it)) {
      const double* row = freq + it.b * d;
      for (int64_t s = 0; s < d; ++s) {
        int prod = 1;
        for (int k = 0; k < n; ++k) prod *= g1[a[k]][it.bd[k]][(s >> (n - 1 - k)) & 1];
        acc += (long double)row[s] * prod;
      }
    }
    e_out[t] = (double)(acc / (long double)xtx_diag(n, a));
  }
  return ORACLE_OK;
}

/* ---- step (ii): eq. (4), one matrix entry at a time ---- */

/* mu[r][c] = sum_i theta_i (Omega_i)[r][c] = 2^{-n} sum_i e_i prod_k sigma_{a_k}[r_k][c_k],
 * visiting for each qubit only the two letters with a nonzero (r_k, c_k) entry
 * (Sec. IV: I,Z share the diagonal pattern, X,Y the off-diagonal one).
 * coef: e_i, length 4^n.  out: interleaved (re, im) per entry. */
int oracle_rho_entries(int n, const double* coef, const int64_t* rows, const int64_t* cols,
                       int64_t nent, double* out) {
  if (n < 1 || n > ORACLE_MAX_N || !coef || !out) return ORACLE_E_ARG;
  int st = ensure_tables();
  if (st) return st;
  int64_t d = (int64_t)1 << n;
  int64_t cnt = rows ? nent : d * d;
  uint64_t ops = 0;
#pragma omp parallel for schedule(static) reduction(+ : ops)
  for (int64_t t = 0; t < cnt; ++t) {
    int64_t r = rows ? rows[t] : t / d, c = rows ? cols[t] : t % d;
    int lt[ORACLE_MAX_N][2], nl[ORACLE_MAX_N];
    int rk[ORACLE_MAX_N], ck[ORACLE_MAX_N];
    for (int k = 0; k < n; ++k) {
      rk[k] = (int)((r >> (n - 1 - k)) & 1);
      ck[k] = (int)((c >> (n - 1 - k)) & 1);
      nl[k] = 0;
      for (int a = 0; a < 4; ++a)
        if (sigma[a][rk[k]][ck[k]] != 0) lt[k][nl[k]++] = a;
    }
    double complex acc = 0;
    int pos[ORACLE_MAX_N];
    for (int k = 0; k < n; ++k) pos[k] = 0;
    for (;;) {
      int64_t i = 0;
      double complex prod = 1;
      for (int k = 0; k < n; ++k) {
        int a = lt[k][pos[k]];
        i = i * 4 + a;
        prod *= sigma[a][rk[k]][ck[k]];
      }
      acc += coef[i] * prod;
      ++ops;
      int k = n - 1;
      while (k >= 0) {
        if (++pos[k] < nl[k]) break;
        pos[k] = 0;
        --k;
      }
      if (k < 0) break;
    }
    acc = acc / (double)d; /* 2^{-n}: exact */
    out[2 * t] = creal(acc);
    out[2 * t + 1] = cimag(acc);
  }
#pragma omp atomic
  ops_step2 += ops;
  return ORACLE_OK;
}

/* Full pipeline on one instance: coefficients (step i) then the whole matrix (step ii). */
int oracle_lre(int n, const uint16_t* counts, uint64_t shots, const uint32_t* nb,
               double* coef, double* rho) {
  int st = oracle_coefs(n, counts, shots, nb, NULL, 0, coef);
  if (st) return st;
  if (rho) st = oracle_rho_entries(n, coef, NULL, NULL, 0, rho);
  return st;
}

void oracle_reset_op_counts(void) { ops_step1 = 0; ops_step2 = 0; }
uint64_t oracle_op_count_step1(void) { return ops_step1; }
uint64_t oracle_op_count_step2(void) { return ops_step2; }

/* ---- reduced operator set (Sec. VI): 4^n product operators instead of 6^n ----
 *
 * The summary of the paper notes that 4^n measured operators instead of the 6^n Pauli
 * projectors suffice (and lower the cost).  The set is not named there; this oracle takes
 * any per-qubit set of four operators E_0..E_3 given by their Pauli components
 *   G[j][a] = Tr(E_j sigma_a),   a = 0..3 (I, X, Y, Z),
 * and the n-qubit operators E_j = (x)_k E_{j_k}, j = sum_k j_k 4^{n-k}.  Eq. (2) gives
 *   Gamma^(j)_i = Tr(E_j Omega_i) = 2^{-n/2} prod_k G[j_k][a_k],
 * so X^T X = sum_j Gamma^(j) Gamma^(j)^T = 2^{-n} (x)_k (G^T G)  (the tensor structure of
 * Sec. III), and eq. (3) is
 *   theta_i = sum_i' (X^T X)^{-1}_{i i'} sum_j p_j Gamma^(j)_{i'},
 * evaluated here term by term over all i' and j (16^n each; fine for n <= 6).
 * (G^T G)^{-1} is the inverse of a 4 x 4 matrix, by Gauss-Jordan elimination with
 * partial pivoting in long double.  p_j = c_j / N with N = sum_j c_j (one setting
 * measures every outcome at once).  Returns e_i = 2^{n/2} theta_i. */

static int inverse4(const long double m_in[4][4], long double inv[4][4]) {
  long double m[4][8];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 8; ++c) m[r][c] = c < 4 ? m_in[r][c] : (long double)(c - 4 == r);
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabsl(m[r][c]) > fabsl(m[piv][c])) piv = r;
    if (fabsl(m[piv][c]) < 1e-12L) return ORACLE_E_ARG;   /* not invertible */
    if (piv != c)
      for (int k = 0; k < 8; ++k) { long double t = m[c][k]; m[c][k] = m[piv][k]; m[piv][k] = t; }
    long double d = m[c][c];
    for (int k = 0; k < 8; ++k) m[c][k] /= d;
    for (int r = 0; r < 4; ++r)
      if (r != c) {
        long double f = m[r][c];
        for (int k = 0; k < 8; ++k) m[r][k] -= f * m[c][k];
      }
  }
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) inv[r][c] = m[r][c + 4];
  return ORACLE_OK;
}

static int povm_coefs_core(int n, const long double* p, const double* G, const int64_t* idx, int64_t nidx,
                           double* e_out);

int oracle_povm_coefs(int n, const uint16_t* counts, const double* G, const int64_t* idx, int64_t nidx,
                      double* e_out) {
  if (n < 1 || n > 8 || !counts || !G || !e_out) return ORACLE_E_ARG;
  int64_t D2 = ipow(4, n);
  uint64_t N = 0;
  for (int64_t j = 0; j < D2; ++j) N += counts[j];
  if (N == 0) return ORACLE_E_EMPTY_BASIS;
  long double* p = (long double*)malloc(sizeof(long double) * (size_t)D2);
  if (!p) return ORACLE_E_ARG;
  for (int64_t j = 0; j < D2; ++j) p[j] = (long double)counts[j] / (long double)N;
  int st = povm_coefs_core(n, p, G, idx, nidx, e_out);
  free(p);
  return st;
}

/* The same with given frequencies p_j (exact probabilities in the pin tests). */
int oracle_povm_coefs_freq(int n, const double* freq, const double* G, const int64_t* idx, int64_t nidx,
                           double* e_out) {
  if (n < 1 || n > 8 || !freq || !G || !e_out) return ORACLE_E_ARG;
  int64_t D2 = ipow(4, n);
  long double* p = (long double*)malloc(sizeof(long double) * (size_t)D2);
  if (!p) return ORACLE_E_ARG;
  for (int64_t j = 0; j < D2; ++j) p[j] = freq[j];
  int st = povm_coefs_core(n, p, G, idx, nidx, e_out);
  free(p);
  return st;
}

static int povm_coefs_core(int n, const long double* p, const double* G, const int64_t* idx, int64_t nidx,
                           double* e_out) {
  int64_t D2 = ipow(4, n);
  long double g[4][4], gtg[4][4], A[4][4];
  for (int j = 0; j < 4; ++j)
    for (int a = 0; a < 4; ++a) g[j][a] = G[4 * j + a];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      gtg[a][b] = 0;
      for (int j = 0; j < 4; ++j) gtg[a][b] += g[j][a] * g[j][b];
    }
  if (inverse4(gtg, A)) return ORACLE_E_ARG;
  /* y_i' = sum_j p_j Gamma^(j)_{i'} * 2^{n/2} (the 2^{-n/2} of Gamma kept aside) */
  long double* y = (long double*)malloc(sizeof(long double) * (size_t)D2);
  if (!y) return ORACLE_E_ARG;
#pragma omp parallel for schedule(static)
  for (int64_t ip = 0; ip < D2; ++ip) {
    int a[ORACLE_MAX_N];
    pauli_digits(n, ip, a);
    long double acc = 0.0L;
    for (int64_t j = 0; j < D2; ++j) {
      int jd[ORACLE_MAX_N];
      pauli_digits(n, j, jd);   /* same base-4 digit order for outcomes */
      long double prod = 1.0L;
      for (int k = 0; k < n; ++k) prod *= g[jd[k]][a[k]];
      acc += p[j] * prod;
    }
    y[ip] = acc;
  }
  /* theta_i = sum_i' (X^T X)^{-1}_{ii'} y_{i'} 2^{-n/2}, (X^T X)^{-1} = 2^n (x) A;
   * e_i = 2^{n/2} theta_i = 2^n sum_i' prod_k A[a_k][a'_k] y_i' */
  int64_t cnt = idx ? nidx : D2;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < cnt; ++t) {
    int64_t i = idx ? idx[t] : t;
    int a[ORACLE_MAX_N];
    pauli_digits(n, i, a);
    long double acc = 0.0L;
    for (int64_t ip = 0; ip < D2; ++ip) {
      int b[ORACLE_MAX_N];
      pauli_digits(n, ip, b);
      long double prod = 1.0L;
      for (int k = 0; k < n; ++k) prod *= A[a[k]][b[k]];
      acc += prod * y[ip];
    }
    e_out[t] = (double)(ldexpl(acc, n));
  }
  free(y);
  return ORACLE_OK;
}

/* Reduced operator set, selected coefficients of eq. (3) without the 4^n-long
 * intermediate: row i of (X^T X)^{-1} = 2^n (x)_k A (A = (G^T G)^{-1}) times
 * Gamma^(j) = 2^{-n/2} (x)_k G[j_k][.] is the product over qubits of the one-qubit
 * row-times-vector sums w[a][j] = sum_a' A[a][a'] G[j][a'] (a Kronecker product times
 * a Kronecker product, taken entry by entry), so
 *   e_i = 2^{n/2} theta_i = 2^n sum_j p_j prod_k w[a_k][j_k],
 * O(n 4^n) per coefficient, for n too large for the full O(16^n) evaluation.
 * cond_out (optional): 2^n sum_j p_j prod_k |w[a_k][j_k]|, the scale against which
 * rounding in any summation order is measured. */
int oracle_povm_coefs_direct(int n, const uint16_t* counts, const double* G, const int64_t* idx, int64_t nidx,
                             double* e_out, double* cond_out) {
  if (n < 1 || n > ORACLE_MAX_N || !counts || !G || !idx || !e_out) return ORACLE_E_ARG;
  int64_t D2 = ipow(4, n);
  uint64_t N = 0;
  for (int64_t j = 0; j < D2; ++j) N += counts[j];
  if (N == 0) return ORACLE_E_EMPTY_BASIS;
  long double g[4][4], gtg[4][4], A[4][4], w[4][4];
  for (int j = 0; j < 4; ++j)
    for (int a = 0; a < 4; ++a) g[j][a] = G[4 * j + a];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) {
      gtg[a][b] = 0;
      for (int j = 0; j < 4; ++j) gtg[a][b] += g[j][a] * g[j][b];
    }
  if (inverse4(gtg, A)) return ORACLE_E_ARG;
  for (int a = 0; a < 4; ++a)
    for (int j = 0; j < 4; ++j) {
      w[a][j] = 0;
      for (int c = 0; c < 4; ++c) w[a][j] += A[a][c] * g[j][c];
    }
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nidx; ++t) {
    int a[ORACLE_MAX_N];
    pauli_digits(n, idx[t], a);
    long double acc = 0.0L, cond = 0.0L;
    for (int64_t j = 0; j < D2; ++j) {
      if (!counts[j]) continue;
      int jd[ORACLE_MAX_N];
      pauli_digits(n, j, jd);
      long double prod = 1.0L;
      for (int k = 0; k < n; ++k) prod *= w[a[k]][jd[k]];
      acc += (long double)counts[j] * prod;
      cond += (long double)counts[j] * fabsl(prod);
    }
    e_out[t] = (double)(ldexpl(acc / (long double)N, n));
    if (cond_out) cond_out[t] = (double)(ldexpl(cond / (long double)N, n));
  }
  return ORACLE_OK;
}
