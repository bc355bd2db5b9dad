"""Seeded synthetic inputs for LRE tomography: states, Born probabilities, counts.

This module is shared by the oracle side (tests, CPU baseline) and the GPU side
(tests, bench).  It simulates the *measurement*, never the estimator: nothing in
here evaluates eq. (3) or eq. (4) of the paper.

Conventions (the same readings the estimator uses; the paper leaves them open):
  * basis b = sum_k b_k 3^{n-k}, b_k in {0: X, 1: Y, 2: Z}, qubit 1 most significant;
  * outcome s = sum_k s_k 2^{n-k}; s_k = 0 is the +1 eigenvector of the measured Pauli.
Counts are uint16 arrays of shape (3^n, 2^n), row b = one measurement setting.
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32_10, philox_counts_rows, philox_counts_rows_fast  # noqa: F401

# Rows of U_b are the bras <psi_{b,s}| of the eigenvectors of sigma_{b+1}, so that
# (U_b psi)_s = <psi_{b,s}|psi> is the amplitude of outcome s.
_R2 = 1.0 / np.sqrt(2.0)
BASIS_BRAS = np.array([
    [[_R2, _R2], [_R2, -_R2]],                 # X: <+|, <-|
    [[_R2, -1j * _R2], [_R2, 1j * _R2]],       # Y: <+i| = (1, -i)/sqrt2, <-i| = (1, i)/sqrt2
    [[1.0, 0.0], [0.0, 1.0]],                  # Z: <0|, <1|
], dtype=np.complex128)


def haar_state(n: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random pure state: normalised complex Gaussian vector of length 2^n."""
    v = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    return v / np.linalg.norm(v)


def ginibre_factor(n: int, rank: int, rng: np.random.Generator) -> np.ndarray:
    """G (2^n x rank) with rho = G G^dagger / Tr(G G^dagger): a rank-`rank` Ginibre state."""
    G = rng.standard_normal((2 ** n, rank)) + 1j * rng.standard_normal((2 ** n, rank))
    return G / np.sqrt(np.real(np.vdot(G.ravel(), G.ravel())))


def rotated_amplitudes(n: int, psi: np.ndarray, b_lo: int = 0, b_hi: int | None = None) -> np.ndarray:
    """(U_b psi)_s for bases b in [b_lo, b_hi): shape (b_hi - b_lo, 2^n), complex128.

    psi may carry extra trailing columns (shape (2^n, r)); then the result has shape
    (b_hi - b_lo, 2^n, r)."""
    B = 3 ** n
    b_hi = B if b_hi is None else b_hi
    psi = np.asarray(psi, dtype=np.complex128)
    extra = psi.shape[1:]
    t = psi.reshape((1,) + (2,) * n + extra)
    # Apply the per-qubit bras axis by axis; the basis axis grows 1 -> 3 -> 9 ...
    for k in range(n):
        # t shape: (3^k, 2,...,2, extra); contract qubit k (axis 1 + k) with U (3, 2, 2)
        t = np.tensordot(BASIS_BRAS, t, axes=([2], [1 + k]))  # (3, 2, 3^k, ...)
        # bring to (3^k, 3, ...) with new outcome axis at position 1 + k
        t = np.moveaxis(t, 2, 0)             # (3^k, 3, 2, rest...)
        t = np.moveaxis(t, 2, 2 + k)         # outcome axis back in qubit k's slot
        t = t.reshape((-1,) + t.shape[2:])   # merge basis axes: b = b_prev * 3 + b_k
    t = t.reshape((B, 2 ** n) + extra)
    return t[b_lo:b_hi]


def born_probs_pure(n: int, psi: np.ndarray) -> np.ndarray:
    """p[b][s] = |<psi_{b,s}|psi>|^2, shape (3^n, 2^n)."""
    return np.abs(rotated_amplitudes(n, psi)) ** 2


def born_probs_mixed(n: int, G: np.ndarray) -> np.ndarray:
    """p[b][s] = <psi_{b,s}| G G^dagger |psi_{b,s}> for rho = G G^dagger (trace one)."""
    A = rotated_amplitudes(n, G)             # (3^n, 2^n, r)
    return np.sum(np.abs(A) ** 2, axis=2)


def ghz_probs(n: int, p_dep: float = 0.0, b_lo: int = 0, b_hi: int | None = None) -> np.ndarray:
    """Probabilities of the n-qubit GHZ state (|0..0> + |1..1>)/sqrt2 under depolarising
    noise: rho = (1 - p) |GHZ><GHZ| + p I / 2^n.  Rows [b_lo, b_hi)."""
    B = 3 ** n
    b_hi = B if b_hi is None else b_hi
    if not 0 <= b_lo <= b_hi <= B:
        raise ValueError("basis range outside [0, 3^n)")
    b = np.arange(b_lo, b_hi)
    digits = np.stack([(b // 3 ** (n - 1 - k)) % 3 for k in range(n)], axis=1)  # (nb, n)
    s = np.arange(2 ** n)
    bits = np.stack([(s >> (n - 1 - k)) & 1 for k in range(n)], axis=1)         # (d, n)
    a0 = np.ones((len(b), 2 ** n), dtype=np.complex128)
    a1 = np.ones((len(b), 2 ** n), dtype=np.complex128)
    for k in range(n):
        u = BASIS_BRAS[digits[:, k]]            # (nb, 2, 2): [s_k][computational]
        a0 *= u[:, bits[:, k], 0]
        a1 *= u[:, bits[:, k], 1]
    p = 0.5 * np.abs(a0 + a1) ** 2
    return (1.0 - p_dep) * p + p_dep / 2 ** n


def multinomial_counts(p: np.ndarray, shots, rng: np.random.Generator) -> np.ndarray:
    """One multinomial draw per basis row: counts[b] ~ Mult(shots_b, p[b]) as uint16.
    `shots` is a scalar or one value per row."""
    p = np.asarray(p, dtype=np.float64)
    p = p / p.sum(axis=1, keepdims=True)
    sh = np.broadcast_to(np.asarray(shots, dtype=np.int64), (p.shape[0],))
    c = rng.multinomial(sh, p)
    if c.max(initial=0) > 65535:
        raise ValueError("a count exceeds the uint16 range")
    return c.astype(np.uint16)


def exact_counts(p: np.ndarray, shots: int) -> np.ndarray:
    """counts = shots * p when that is integral for every entry (stabiliser states with
    2^n dividing shots); raises otherwise."""
    c = np.asarray(p, dtype=np.float64) * shots
    r = np.rint(c)
    if np.max(np.abs(c - r)) > 1e-9:
        raise ValueError("shots * p is not integral")
    return r.astype(np.uint16)


def maximally_mixed_counts(n: int, per_outcome: int) -> np.ndarray:
    """Every outcome of every basis observed `per_outcome` times (the paper's test state)."""
    return np.full((3 ** n, 2 ** n), per_outcome, dtype=np.uint16)
