"""Pins of the CPU oracle against facts fixed by the paper and by the mathematics.

None of these tests compares the oracle with itself: every expected value comes
from the paper's printed one-qubit case, from closed forms, from brute-force least
squares with explicit matrices (tests/refs.py), or from exact-recovery identities.
"""
import os

import numpy as np
import pytest

import oracle
import tomo_inputs as ti
from tests import refs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_gamma():
    rows, xtx = [], None
    with open(os.path.join(GOLDEN, "one_qubit_gamma.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "gamma":
                rows.append([float(v) for v in parts[2:]])
            elif parts[0] == "xtx_diag":
                xtx = np.diag([float(v) for v in parts[1:]])
    return np.array(rows) / np.sqrt(2.0), xtx


def test_one_qubit_tables_match_printed_case():
    """Sec. III one-qubit case: the six Gamma vectors and X^T X = diag{3,1,1,1}."""
    gamma, xtx = oracle.one_qubit_tables()
    g_ref, x_ref = _golden_gamma()
    np.testing.assert_allclose(gamma, g_ref, atol=1e-15)
    np.testing.assert_array_equal(xtx, x_ref)


@pytest.mark.parametrize("c", [(7, 3, 2, 8, 10, 0), (1, 0, 0, 1, 5, 5), (12, 13, 1, 24, 25, 0)])
def test_one_qubit_hand_case(c):
    """n = 1 by hand: e = (1, (c0-c1)/N_X, (c2-c3)/N_Y, (c4-c5)/N_Z) and
    mu = (1/2)[[1+e_Z, e_X - i e_Y], [e_X + i e_Y, 1 - e_Z]] (Bloch form)."""
    counts = np.array(c, dtype=np.uint16).reshape(3, 2)
    N = counts.sum(axis=1)
    e, mu = oracle.lre(1, counts, 0)
    ex = [1.0, (c[0] - c[1]) / N[0], (c[2] - c[3]) / N[1], (c[4] - c[5]) / N[2]]
    np.testing.assert_allclose(e, ex, rtol=0, atol=1e-16)
    mu_ref = 0.5 * np.array([[1 + ex[3], ex[1] - 1j * ex[2]], [ex[1] + 1j * ex[2], 1 - ex[3]]])
    np.testing.assert_allclose(mu, mu_ref, rtol=0, atol=1e-16)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_bruteforce_least_squares(n):
    """Eq. (3) with the explicit 6^n x 4^n design matrix, solved by numpy.linalg.lstsq,
    equals the oracle's sparse evaluation; eq. (4) as an explicit sum of Kronecker
    products equals the oracle's mu."""
    rng = np.random.default_rng(100 + n)
    psi = ti.haar_state(n, rng)
    counts = ti.multinomial_counts(ti.born_probs_pure(n, psi), 500, rng)
    freq = counts / counts.sum(axis=1, keepdims=True)
    e_ls, mu_ls = refs.lstsq_estimate(n, freq)
    e, mu = oracle.lre(n, counts, 500)
    np.testing.assert_allclose(e, e_ls, rtol=0, atol=1e-12)
    np.testing.assert_allclose(mu, mu_ls, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_exact_recovery_from_projector_probabilities(n):
    """Noise-free frequencies Tr(rho P_j) from explicit projectors: least squares is exact
    (X has full column rank), so the estimate returns rho and its Pauli expectations."""
    rng = np.random.default_rng(200 + n)
    G = ti.ginibre_factor(n, 2, rng)
    rho = G @ G.conj().T
    p = refs.born_from_projectors(n, rho)
    e = oracle.coefs_freq(n, p)
    np.testing.assert_allclose(e, refs.true_expectations(n, rho), rtol=0, atol=1e-13)
    mu = oracle.rho(n, e)
    np.testing.assert_allclose(mu, rho, rtol=0, atol=1e-14)


@pytest.mark.parametrize("n", [5, 6])
def test_exact_recovery_generator_probabilities(n):
    """Same identity at larger n with the generator's Born probabilities: a pure state
    comes back as itself."""
    rng = np.random.default_rng(300 + n)
    psi = ti.haar_state(n, rng)
    e = oracle.coefs_freq(n, ti.born_probs_pure(n, psi))
    mu = oracle.rho(n, e)
    np.testing.assert_allclose(mu, np.outer(psi, psi.conj()), rtol=0, atol=1e-13)


@pytest.mark.parametrize("n", [1, 3, 5])
def test_maximally_mixed_is_exact(n):
    """The paper's own test state (Sec. IV): equal counts in every outcome give e_i = 0
    for i != 0, e_0 = 1 and mu = I / 2^n, exactly."""
    K = 3
    counts = ti.maximally_mixed_counts(n, K)
    e, mu = oracle.lre(n, counts, K * 2 ** n)
    assert e[0] == 1.0
    assert np.all(e[1:] == 0.0)
    assert np.array_equal(mu, np.eye(2 ** n) / 2 ** n)


@pytest.mark.parametrize("n,p_dep", [(2, 0.0), (3, 0.0), (4, 0.0), (3, 0.5), (5, 0.5)])
def test_ghz_closed_form(n, p_dep):
    """GHZ (optionally half depolarised) with shots a multiple of 2^(n+1): every count is
    shots * p exactly, so the estimate equals the closed-form expectations exactly."""
    shots = 4 * 2 ** (n + 1)
    counts = ti.exact_counts(ti.ghz_probs(n, p_dep), shots)
    e, mu = oracle.lre(n, counts, shots)
    np.testing.assert_array_equal(e, refs.ghz_expectations(n, p_dep))
    np.testing.assert_allclose(mu, refs.ghz_density(n, p_dep), rtol=0, atol=1e-15)


def test_ghz3_nonzero_set():
    """n = 3 GHZ: exactly 8 nonzero Pauli expectations, III IZZ ZIZ ZZI XXX = +1 and
    XYY YXY YYX = -1."""
    shots = 64
    e = oracle.coefs(3, ti.exact_counts(ti.ghz_probs(3), shots), shots)
    letters = {"I": 0, "X": 1, "Y": 2, "Z": 3}
    idx = lambda w: sum(letters[ch] * 4 ** (2 - k) for k, ch in enumerate(w))
    want = {idx(w): 1.0 for w in ["III", "IZZ", "ZIZ", "ZZI", "XXX"]}
    want.update({idx(w): -1.0 for w in ["XYY", "YXY", "YYX"]})
    nz = {i: v for i, v in enumerate(e) if v != 0}
    assert nz == want


@pytest.mark.parametrize("n", [3, 4, 5])
def test_invariants_multinomial(n):
    """Unit trace, Hermiticity and |e_i| <= 1 on noisy data (Sec. II: mu is Hermitian with
    Tr mu = 1; it need not be positive)."""
    rng = np.random.default_rng(400 + n)
    psi = ti.haar_state(n, rng)
    counts = ti.multinomial_counts(ti.born_probs_pure(n, psi), 300, rng)
    e, mu = oracle.lre(n, counts, 300)
    assert e[0] == 1.0
    assert np.all(np.abs(e) <= 1.0)
    assert abs(np.trace(mu) - 1.0) < 1e-13
    assert np.max(np.abs(mu - mu.conj().T)) == 0.0


def test_per_basis_path_equals_uniform_when_totals_agree():
    n = 4
    rng = np.random.default_rng(7)
    counts = ti.multinomial_counts(ti.born_probs_pure(n, ti.haar_state(n, rng)), 777, rng)
    e_u = oracle.coefs(n, counts, 777)
    e_b = oracle.coefs(n, counts, 0)
    e_nb = oracle.coefs(n, counts, 0, np.full(3 ** n, 777, dtype=np.uint32))
    np.testing.assert_allclose(e_b, e_u, rtol=0, atol=2e-16)
    np.testing.assert_array_equal(e_b, e_nb)


def test_unequal_shots_match_bruteforce():
    """Per-basis totals (reading: p_j = c / N_b within each basis) against brute-force LS."""
    n = 3
    rng = np.random.default_rng(8)
    p = ti.born_probs_pure(n, ti.haar_state(n, rng))
    shots = rng.integers(50, 400, size=3 ** n)
    counts = ti.multinomial_counts(p, shots, rng)
    freq = counts / counts.sum(axis=1, keepdims=True)
    e_ls, mu_ls = refs.lstsq_estimate(n, freq)
    e, mu = oracle.lre(n, counts, 0)
    np.testing.assert_allclose(e, e_ls, rtol=0, atol=1e-12)
    np.testing.assert_allclose(mu, mu_ls, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_operation_counts(n):
    """Sec. III: dropping the zero terms leaves 12^n terms in step (i) and 8^n in step (ii)."""
    counts = ti.maximally_mixed_counts(n, 1)
    oracle.reset_op_counts()
    oracle.lre(n, counts, 2 ** n)
    assert oracle.op_counts() == (12 ** n, 8 ** n)


def test_integer_sums_and_single_division():
    """With uniform shots e_i is the correctly rounded quotient T_i / (3^(n-w) shots)."""
    n = 4
    rng = np.random.default_rng(9)
    counts = ti.multinomial_counts(ti.born_probs_pure(n, ti.haar_state(n, rng)), 999, rng)
    T = oracle.pauli_sums(n, counts)
    e = oracle.coefs(n, counts, 999)
    w = np.array([refs.pauli_weight(n, i) for i in range(4 ** n)])
    from fractions import Fraction
    for i in range(4 ** n):
        exact = Fraction(int(T[i]), 3 ** (n - int(w[i])) * 999)
        assert e[i] == float(exact)  # float(Fraction) rounds correctly
    # brute-force check of the integer numerators at a few coefficients
    for i in [0, 1, 5, 27, 255]:
        a = [(i // 4 ** (n - 1 - k)) % 4 for k in range(n)]
        tot = 0
        for b in range(3 ** n):
            bd = [(b // 3 ** (n - 1 - k)) % 3 for k in range(n)]
            if any(a[k] and a[k] != bd[k] + 1 for k in range(n)):
                continue
            for s in range(2 ** n):
                sgn = 1
                for k in range(n):
                    if a[k] and (s >> (n - 1 - k)) & 1:
                        sgn = -sgn
                tot += sgn * int(counts[b, s])
        assert tot == T[i]


def test_maximally_mixed_mse_closed_form():
    """Sec. V: for the maximally mixed state the mean squared HS distance of mu is
    (5/6)^n / N_0 to leading order; with multinomial counts the exact value is
    (10^n - 1) / (6^n * shots) = ((5/6)^n - 12^-n) / N_0 with N_0 = shots / 2^n.
    Monte Carlo over 600 seeded repetitions, checked within 4 standard errors."""
    n, shots, reps = 3, 64, 600
    d = 2 ** n
    p = np.full((3 ** n, d), 1.0 / d)
    rng = np.random.default_rng(1602)
    hs = np.empty(reps)
    for t in range(reps):
        counts = ti.multinomial_counts(p, shots, rng)
        _, mu = oracle.lre(n, counts, shots)
        hs[t] = np.sum(np.abs(mu - np.eye(d) / d) ** 2)
    exact = (10 ** n - 1) / (6 ** n * shots)
    N0 = shots / d
    assert abs(exact - ((5 / 6) ** n - 12.0 ** -n) / N0) < 1e-15
    se = hs.std(ddof=1) / np.sqrt(reps)
    assert abs(hs.mean() - exact) < 4 * se, (hs.mean(), exact, se)


def test_error_paths():
    counts = ti.maximally_mixed_counts(2, 2)
    with pytest.raises(oracle.OracleError):
        oracle.coefs(2, counts, 9)  # rows sum to 8
    bad = counts.copy()
    bad[3] = 0
    with pytest.raises(oracle.OracleError):
        oracle.coefs(2, bad, 0)     # empty basis
    with pytest.raises(ValueError):
        oracle.coefs(2, counts[:4], 8)


def test_coef_from_rows_matches_full():
    n = 4
    rng = np.random.default_rng(11)
    shots = rng.integers(100, 300, size=3 ** n)
    counts = ti.multinomial_counts(ti.born_probs_pure(n, ti.haar_state(n, rng)), shots, rng)
    e = oracle.coefs(n, counts, 0)
    for i in [0, 3, 17, 100, 255]:
        bases = oracle.compatible_bases(n, i)
        assert len(bases) == 3 ** (n - refs.pauli_weight(n, i))
        v = oracle.coef_from_rows(n, i, counts[bases], counts[bases].sum(axis=1))
        assert v == e[i]


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_basis_sums_bruteforce(n):
    """Per-basis signed sums of eq. (3) (the part sum_s c[b][s] 2^{n/2} gamma_i^(b,s) of one
    setting, Sec. III): the oracle against a brute-force sum over every outcome with the
    sign (-1)^popcount(s & m), m the support of i, for every (basis, coefficient) pair.
    Compatibility (letter a_k = b_k + 1 wherever a_k is not I) and the support mask are
    derived here from digit arrays, independently of the oracle's own decoding; pairs
    that are not compatible must give 0 (their Gamma entries vanish)."""
    rng = np.random.default_rng(200 + n)
    counts = rng.integers(0, 1000, size=(3 ** n, 2 ** n)).astype(np.uint16)
    b = np.repeat(np.arange(3 ** n), 4 ** n)
    i = np.tile(np.arange(4 ** n), 3 ** n)
    # digit p counts from the least significant position (qubit n - p in the paper's order)
    bd = np.stack([(b // 3 ** p) % 3 for p in range(n)], axis=1)
    ad = np.stack([(i >> (2 * p)) & 3 for p in range(n)], axis=1)
    compat = np.all((ad == 0) | (ad == bd + 1), axis=1)
    m = np.sum((ad != 0) * (1 << np.arange(n)), axis=1)
    s = np.arange(2 ** n)
    par = np.array([bin(v).count("1") & 1 for v in range(2 ** n)])
    sign = 1 - 2 * par[np.bitwise_and.outer(m, s)]                # (pairs, 2^n)
    S = np.sum(counts[b].astype(np.int64) * sign, axis=1)
    S[~compat] = 0
    got = oracle.basis_sums(n, counts, b, i)
    np.testing.assert_array_equal(got, S)
    assert np.count_nonzero(compat) == 6 ** n                    # 2^n supports per basis


def _all_pairs(n, idx):
    pr, pc, ps = [], [], []
    for t, i in enumerate(idx):
        b = oracle.compatible_bases(n, int(i))
        pr.append(b)
        pc.append(np.full(len(b), i))
        ps.append(np.full(len(b), t))
    return np.concatenate(pr), np.concatenate(pc), np.concatenate(ps)


@pytest.mark.parametrize("n,p_dep", [(3, 0.0), (5, 0.5)])
def test_accumulate_pairs_ghz_closed_form(n, p_dep):
    """Streaming eq. (3) (rows visited in chunks, pairs in an arbitrary order) on exact
    GHZ counts reproduces the closed-form Pauli expectations."""
    shots = 2 ** (n + 1)
    counts = ti.exact_counts(ti.ghz_probs(n, p_dep), shots)
    idx = np.arange(4 ** n)
    pr, pc, ps = _all_pairs(n, idx)
    order = np.random.default_rng(n).permutation(len(pr))
    pr, pc, ps = pr[order], pc[order], ps[order]
    acc = np.zeros(len(idx), dtype=np.longdouble)
    chunk = 7
    for b0 in range(0, 3 ** n, chunk):
        bases = np.arange(b0, min(3 ** n, b0 + chunk))
        sel = (pr >= b0) & (pr < b0 + chunk)
        oracle.accumulate_pairs(n, counts[bases], bases, counts[bases].sum(axis=1),
                                pr[sel] - b0, pc[sel], ps[sel], acc)
    e = oracle.coef_from_acc(n, idx, acc)
    np.testing.assert_allclose(e, refs.ghz_expectations(n, p_dep), rtol=0, atol=1e-15)


def test_accumulate_pairs_bruteforce_least_squares():
    """Streaming eq. (3) with unequal per-basis totals equals the explicit 6^n x 4^n
    least-squares solution (numpy.linalg.lstsq) at n = 3."""
    n = 3
    rng = np.random.default_rng(33)
    shots = rng.integers(50, 400, size=3 ** n)
    counts = ti.multinomial_counts(ti.born_probs_pure(n, ti.haar_state(n, rng)), shots, rng)
    freq = (counts / counts.sum(axis=1, keepdims=True)).ravel()
    e_ls, _ = refs.lstsq_estimate(n, freq)
    idx = np.arange(4 ** n)
    pr, pc, ps = _all_pairs(n, idx)
    acc = np.zeros(len(idx), dtype=np.longdouble)
    oracle.accumulate_pairs(n, counts, np.arange(3 ** n), counts.sum(axis=1), pr, pc, ps, acc)
    assert np.max(np.abs(oracle.coef_from_acc(n, idx, acc) - e_ls)) <= 1e-12


def test_accumulate_pairs_errors():
    n = 2
    counts = ti.maximally_mixed_counts(n, 3)
    acc = np.zeros(4, dtype=np.longdouble)
    with pytest.raises(oracle.OracleError):       # declared total differs from the row
        oracle.accumulate_pairs(n, counts, np.arange(9), np.full(9, 11), [0], [0], [0], acc)
    with pytest.raises(oracle.OracleError):       # row index outside the chunk
        oracle.accumulate_pairs(n, counts, np.arange(9), np.full(9, 12), [9], [0], [0], acc)
