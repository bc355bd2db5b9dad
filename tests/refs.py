"""Small, explicit-matrix references used to pin the oracle (tests only).

Everything here is built from dense matrices with numpy.kron, independently of
oracle/lre_oracle.c: the Pauli matrices of Sec. III, the representation basis of
eq. (5), the eigenprojectors of local Pauli measurements, the design matrix X of
eq. (3) and the matrix sum of eq. (4).  Sizes are exponential, so n <= 4.
"""
from __future__ import annotations

import numpy as np

SIGMA = [np.eye(2, dtype=np.complex128),
         np.array([[0, 1], [1, 0]], dtype=np.complex128),
         np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
         np.array([[1, 0], [0, -1]], dtype=np.complex128)]


def kron_all(mats):
    out = np.ones((1, 1), dtype=np.complex128)
    for m in mats:
        out = np.kron(out, m)
    return out


def omega(n, i):
    """Omega_i = 2^{-n/2} (x)_k sigma_{i_k}, i = sum_k i_k 4^{n-k}  (eq. 5)."""
    digits = [(i // 4 ** (n - 1 - k)) % 4 for k in range(n)]
    return kron_all([SIGMA[a] for a in digits]) / 2 ** (n / 2)


def projector(n, b, s):
    """Eigenprojector of the local Pauli setting b (letters X,Y,Z = 0,1,2) for outcome s
    (bit 0 = eigenvalue +1): (x)_k (I + (-1)^{s_k} sigma_{b_k+1}) / 2, built from the
    eigenvectors, not from the formula used by the oracle."""
    vecs = {
        (0, 0): np.array([1, 1]) / np.sqrt(2), (0, 1): np.array([1, -1]) / np.sqrt(2),
        (1, 0): np.array([1, 1j]) / np.sqrt(2), (1, 1): np.array([1, -1j]) / np.sqrt(2),
        (2, 0): np.array([1, 0]), (2, 1): np.array([0, 1]),
    }
    mats = []
    for k in range(n):
        bk = (b // 3 ** (n - 1 - k)) % 3
        sk = (s >> (n - 1 - k)) & 1
        v = vecs[(bk, sk)].astype(np.complex128)
        mats.append(np.outer(v, v.conj()))
    return kron_all(mats)


def design_matrix(n):
    """X with rows Gamma^(j) = (Tr(P_j Omega_i))_i, j = (b, s) in row-major order."""
    d = 2 ** n
    Om = np.stack([omega(n, i) for i in range(4 ** n)])            # (4^n, d, d)
    rows = []
    for b in range(3 ** n):
        for s in range(d):
            P = projector(n, b, s)
            rows.append(np.real(np.einsum("rc,icr->i", P, Om)))
    return np.array(rows)


def lstsq_estimate(n, freq):
    """Least squares of eq. (3) by brute force: argmin ||X theta - p||.  Returns the Pauli
    expectations e = 2^{n/2} theta and mu = sum_i theta_i Omega_i (eq. 4)."""
    X = design_matrix(n)
    theta, *_ = np.linalg.lstsq(X, np.asarray(freq, dtype=np.float64).ravel(), rcond=None)
    mu = sum(theta[i] * omega(n, i) for i in range(4 ** n))
    return theta * 2 ** (n / 2), mu


def born_from_projectors(n, rho):
    """p[b][s] = Tr(rho P_{b,s}) from explicit projectors."""
    d = 2 ** n
    p = np.zeros((3 ** n, d))
    for b in range(3 ** n):
        for s in range(d):
            p[b, s] = np.real(np.trace(rho @ projector(n, b, s)))
    return p


def true_expectations(n, rho):
    """Tr(rho (x)_k sigma_{a_k}) for every Pauli index."""
    return np.array([np.real(np.trace(rho @ omega(n, i))) * 2 ** (n / 2) for i in range(4 ** n)])


def ghz_expectations(n, p_dep=0.0):
    """Closed form for rho = (1-p)|GHZ_n><GHZ_n| + p I/2^n:  the Pauli string over {I,Z}
    with an even number of Z has expectation 1; a string over {X,Y} with an even number
    of Y has (-1)^{#Y/2}; every other string 0.  Non-identity values scale by (1-p)."""
    i = np.arange(4 ** n)
    letters = np.stack([(i >> (2 * (n - 1 - k))) & 3 for k in range(n)], axis=1)
    nz = np.sum(letters == 3, axis=1)
    ny = np.sum(letters == 2, axis=1)
    iz = np.all((letters == 0) | (letters == 3), axis=1) & (nz % 2 == 0)
    xy = np.all((letters == 1) | (letters == 2), axis=1) & (ny % 2 == 0)
    out = np.zeros(4 ** n)
    out[iz] = 1.0
    out[xy] = np.where((ny[xy] // 2) % 2 == 0, 1.0, -1.0)
    out[1:] *= (1.0 - p_dep)
    return out


def ghz_density(n, p_dep=0.0):
    d = 2 ** n
    psi = np.zeros(d, dtype=np.complex128)
    psi[0] = psi[-1] = 1 / np.sqrt(2)
    return (1 - p_dep) * np.outer(psi, psi.conj()) + p_dep * np.eye(d) / d


def pauli_weight(n, i):
    return sum(1 for k in range(n) if (i // 4 ** k) % 4 != 0)
