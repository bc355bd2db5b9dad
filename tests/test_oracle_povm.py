"""Pins of the oracle for the reduced operator set (4^n product operators, Sec. VI)
against facts fixed independently of it: least squares with the explicit design matrix
built from dense operators (numpy.kron, numpy.linalg.lstsq), exact recovery of a state
from its exact outcome probabilities, and the maximally mixed state.

Two per-qubit operator sets are used: the tetrahedral informationally complete POVM
E_j = (I + r_j . sigma) / 4 (a 4-outcome measurement of one setting), and four of the
six Pauli eigenprojectors {Z+, Z-, X+, Y+} (linearly independent, not a POVM)."""
import numpy as np
import pytest

import oracle
from tests import refs

TET = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]]) / np.sqrt(3.0)


def tetra_ops():
    return [0.25 * (refs.SIGMA[0] + sum(r[a] * refs.SIGMA[a + 1] for a in range(3))) for r in TET]


def pauli_subset_ops():
    z0 = np.array([1, 0], dtype=complex)
    z1 = np.array([0, 1], dtype=complex)
    xp = np.array([1, 1], dtype=complex) / np.sqrt(2)
    yp = np.array([1, 1j], dtype=complex) / np.sqrt(2)
    return [np.outer(v, v.conj()) for v in (z0, z1, xp, yp)]


def components(ops):
    """G[j][a] = Tr(E_j sigma_a) (real for Hermitian E_j)."""
    return np.array([[np.trace(E @ refs.SIGMA[a]).real for a in range(4)] for E in ops])


def nqubit_op(ops, n, j):
    digits = [(j // 4 ** (n - 1 - k)) % 4 for k in range(n)]
    return refs.kron_all([ops[d] for d in digits])


def design(ops, n):
    Om = np.stack([refs.omega(n, i) for i in range(4 ** n)])
    return np.array([np.real(np.einsum("rc,icr->i", nqubit_op(ops, n, j), Om)) for j in range(4 ** n)])


def ginibre(n, rank, rng):
    g = rng.normal(size=(2 ** n, rank)) + 1j * rng.normal(size=(2 ** n, rank))
    r = g @ g.conj().T
    return r / np.trace(r).real


@pytest.mark.parametrize("which", ["tetra", "pauli_subset"])
@pytest.mark.parametrize("n", [1, 2, 3])
def test_povm_bruteforce_least_squares(which, n):
    ops = tetra_ops() if which == "tetra" else pauli_subset_ops()
    rng = np.random.default_rng(40 + n)
    X = design(ops, n)
    p = rng.uniform(0.01, 1.0, size=4 ** n)
    p /= p.sum()
    theta, *_ = np.linalg.lstsq(X, p, rcond=None)
    e_ls = theta * 2 ** (n / 2)
    e = oracle.povm_coefs_freq(n, p, components(ops))
    assert np.max(np.abs(e - e_ls)) <= 1e-12


@pytest.mark.parametrize("n", [1, 2, 3, 4])
def test_povm_exact_recovery(n):
    """Exact probabilities p_j = Tr(rho E_j) give back every Pauli expectation of rho."""
    ops = tetra_ops()
    rng = np.random.default_rng(50 + n)
    rho = ginibre(n, 2, rng)
    p = np.array([np.trace(rho @ nqubit_op(ops, n, j)).real for j in range(4 ** n)])
    assert abs(p.sum() - 1) < 1e-12                        # a complete POVM
    e_true = np.array([np.trace(rho @ refs.omega(n, i)).real * 2 ** (n / 2) for i in range(4 ** n)])
    e = oracle.povm_coefs_freq(n, p, components(ops))
    assert np.max(np.abs(e - e_true)) <= 1e-12
    assert abs(e[0] - 1) <= 1e-13


def test_povm_counts_maximally_mixed_and_frequencies():
    ops = tetra_ops()
    G = components(ops)
    n = 3
    c = np.full(4 ** n, 7, dtype=np.uint16)
    e = oracle.povm_coefs(n, c, G)
    assert abs(e[0] - 1) <= 1e-14 and np.max(np.abs(e[1:])) <= 1e-14
    rng = np.random.default_rng(3)
    c = rng.integers(0, 50, size=4 ** n).astype(np.uint16)
    # counts: p = c / N formed in long double; the frequencies here are binary64 quotients
    assert np.max(np.abs(oracle.povm_coefs(n, c, G) - oracle.povm_coefs_freq(n, c / c.sum(), G))) <= 1e-15
    idx = np.array([0, 5, 63])
    np.testing.assert_array_equal(oracle.povm_coefs(n, c, G, idx=idx), oracle.povm_coefs(n, c, G)[idx])


def test_povm_errors():
    G = components(tetra_ops())
    G[3] = G[2]                                           # two equal operators: not informationally complete
    with pytest.raises(oracle.OracleError):
        oracle.povm_coefs(2, np.ones(16, dtype=np.uint16), G)
    with pytest.raises(oracle.OracleError):
        oracle.povm_coefs(2, np.zeros(16, dtype=np.uint16), components(tetra_ops()))


@pytest.mark.parametrize("which", ["tetra", "pauli_subset"])
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_povm_direct_matches_full(which, n):
    """The selected-coefficient entry (entrywise Kronecker row times Gamma^(j)) equals the
    full evaluation, which the least-squares pins above fix; its scale bounds |e|."""
    G = components(tetra_ops() if which == "tetra" else pauli_subset_ops())
    rng = np.random.default_rng(60 + n)
    c = rng.integers(0, 300, size=4 ** n).astype(np.uint16)
    idx = np.arange(4 ** n)
    e_full = oracle.povm_coefs(n, c, G)
    e, cond = oracle.povm_coefs_direct(n, c, G, idx)
    assert np.max(np.abs(e - e_full) / np.maximum(cond, 1.0)) <= 1e-14
    assert np.all(np.abs(e) <= cond * (1 + 1e-14))
    if which == "tetra":                 # a complete POVM: the frequencies fix the trace
        assert abs(e[0] - 1) <= 1e-14


def test_povm_direct_exact_recovery_product_state():
    """A product state measured with the tetrahedral POVM: outcome probabilities factor,
    and with the Bloch vector (sqrt3/4, 0, 0) on every qubit each one-qubit probability is
    5/16 or 3/16, so counts 5^m 3^(n-m) are exact; e_i = prod_k (Bloch vector components),
    i.e. 1 for I, sqrt3/4 for X and 0 for Y, Z letters."""
    n = 6
    G = components(tetra_ops())
    j = np.arange(4 ** n)
    m = np.zeros(4 ** n, dtype=np.int64)
    for k in range(n):
        m += ((j >> (2 * k)) & 3) < 2        # outcomes 0, 1 of the frame have r_x = +1
    c = (5 ** m * 3 ** (n - m)).astype(np.uint16)
    rng = np.random.default_rng(6)
    idx = np.concatenate([[0], rng.integers(0, 4 ** n, 200)])
    e, _ = oracle.povm_coefs_direct(n, c, G, idx)
    want = np.ones(len(idx))
    for k in range(n):
        a = (idx >> (2 * k)) & 3
        want *= np.where(a == 0, 1.0, np.where(a == 1, np.sqrt(3) / 4, 0.0))
    assert np.max(np.abs(e - want)) <= 1e-14
