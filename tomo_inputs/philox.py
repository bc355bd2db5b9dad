"""Philox4x32-10 counter-based generator (numpy twin of the on-device generator).

Written from the published definition (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit
key; each of the 10 rounds multiplies counter words 0 and 2 by two fixed odd
constants (64-bit products split into high and low halves), mixes the high halves
with the other two counter words and the key, and the key is bumped by two Weyl
increments between rounds.

Count tensor recipe used for the 14-qubit workload: for basis b and outcome s,
    x = Philox4x32-10(counter = (s, b mod 2^32, b >> 32, 0), key = (seed mod 2^32, seed >> 32))
    c[b][s] = (x[0] * 13) >> 32          (uniform on {0, ..., 12})
The HIP generator in ``philox_gen.hip`` implements the same recipe; tests compare
the two bit for bit.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
COUNT_LEVELS = 13  # counts uniform on {0, ..., 12}


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  All arguments are broadcastable uint32 arrays; returns
    the four output words as uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint32).astype(np.uint64)
    c1 = np.asarray(c1, dtype=np.uint32).astype(np.uint64)
    c2 = np.asarray(c2, dtype=np.uint32).astype(np.uint64)
    c3 = np.asarray(c3, dtype=np.uint32).astype(np.uint64)
    k0 = np.asarray(k0, dtype=np.uint32).astype(np.uint64)
    k1 = np.asarray(k1, dtype=np.uint32).astype(np.uint64)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(W0)) & MASK
            k1 = (k1 + np.uint64(W1)) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32), c2.astype(np.uint32),
            c3.astype(np.uint32))


def philox_counts_rows(n: int, seed: int, bases) -> np.ndarray:
    """Count rows c[b][:] of the 14-qubit-style Philox workload for the given bases.
    Returns uint16 array (len(bases), 2^n)."""
    b = np.asarray(bases, dtype=np.uint64).reshape(-1, 1)
    s = np.arange(2 ** n, dtype=np.uint64).reshape(1, -1)
    k0 = np.uint32(seed & 0xFFFFFFFF)
    k1 = np.uint32((seed >> 32) & 0xFFFFFFFF)
    x0, _, _, _ = philox4x32_10(s.astype(np.uint32), (b & MASK).astype(np.uint32),
                                (b >> np.uint64(32)).astype(np.uint32), np.uint32(0), k0, k1)
    c = (x0.astype(np.uint64) * np.uint64(COUNT_LEVELS)) >> np.uint64(32)
    return c.astype(np.uint16)


_clib = None


def philox_counts_rows_fast(n: int, seed: int, bases, paired: bool = False) -> tuple[np.ndarray, np.ndarray]:
    """Same rows as philox_counts_rows, from the OpenMP C twin; also returns the row totals.
    paired: outcome 2k + 1 becomes 12 minus outcome 2k (uniform totals 12 * 2^(n-1)).
    Builds the C twin on first use."""
    global _clib
    import ctypes
    if _clib is None:
        from .build import build_cpu
        L = ctypes.CDLL(build_cpu(force=False))
        L.tomo_philox_rows_mode.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.tomo_philox_rows_mode.restype = ctypes.c_int
        _clib = L
    b = np.ascontiguousarray(bases, dtype=np.int64)
    out = np.empty((len(b), 2 ** n), dtype=np.uint16)
    nb = np.empty(len(b), dtype=np.uint32)
    rc = _clib.tomo_philox_rows_mode(n, seed, b.ctypes.data, len(b), out.ctypes.data, nb.ctypes.data,
                                     1 if paired else 0)
    if rc:
        raise RuntimeError("tomo_philox_rows failed")
    return out, nb
