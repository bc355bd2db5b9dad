"""Oracle for step (iii) of LRE: the physical density matrix closest to mu (test
infrastructure only, like the rest of ``oracle/``).

Sec. II, step (iii): mu may have negative eigenvalues; the estimate rho is the density
matrix closest to mu, found with the fast algorithm the paper cites (Smolin, Gambetta
and Smith, 2012).  Written from that algorithm's statement:

1. eigendecompose mu = V diag(m) V^H (a library eigensolver, ``numpy.linalg.eigh``);
2. walk the eigenvalues from the smallest up with a running sum a of the removed mass:
   while the current one plus a shared over the k eigenvalues still kept is negative,
   set it to 0 and add it to a; every eigenvalue kept is then raised by a / k;
3. rho = V diag(lambda) V^H.

Unlike the C oracle this module is plain numpy: the only library primitives are the
eigensolver and a matrix product.
"""
from __future__ import annotations

import numpy as np


def truncate_spectrum(m: np.ndarray) -> np.ndarray:
    """Step 2 on eigenvalues `m` (any order; the trace is kept): returns lambda >= 0 in
    the same order, summing to sum(m)."""
    m = np.asarray(m, dtype=np.float64)
    order = np.argsort(m)               # ascending
    lam = np.zeros_like(m)
    a = 0.0
    k = m.size                          # eigenvalues still kept
    i = 0
    while i < m.size and m[order[i]] + a / k < 0.0:
        a += m[order[i]]
        k -= 1
        i += 1
    for j in range(i, m.size):
        lam[order[j]] = m[order[j]] + a / k
    return lam


def project(mu: np.ndarray):
    """rho closest to the Hermitian mu (trace 1): returns (rho, eigenvalues of mu
    ascending, lambda ascending)."""
    mu = np.asarray(mu, dtype=np.complex128)
    m, V = np.linalg.eigh(mu)
    lam = truncate_spectrum(m)
    rho = (V * lam) @ V.conj().T
    return rho, m, lam
