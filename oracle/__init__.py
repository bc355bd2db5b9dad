"""Plain CPU oracle for LRE tomography (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path never does: it runs on
the HIP library and fails loudly when that library is missing.

The arithmetic lives in ``lre_oracle.c`` (plain C, OpenMP over output entries,
int64 for integer sums, binary64 / long double otherwise); this module only
marshals numpy arrays through ctypes.  See the header of ``lre_oracle.c`` for the
paper passages each function follows (Sec. II eqs. 2-4, Sec. III eq. 5 and the
one-qubit worked case).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lre_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

GCC_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
             "-fno-fast-math"]

STATUS = {0: "ok", 1: "bad argument", 2: "row sum differs from the declared shots",
          3: "basis with zero counts", 4: "one-qubit tables not integral"}


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile lre_oracle.c with gcc into liboracle.so (next to the source)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_one_qubit_tables.argtypes = [P, P]
        lib.oracle_pauli_sums.argtypes = [ctypes.c_int, P, P, I64, P]
        lib.oracle_basis_sums.argtypes = [ctypes.c_int, P, P, P, I64, P]
        lib.oracle_coefs.argtypes = [ctypes.c_int, P, ctypes.c_uint64, P, P, I64, P]
        lib.oracle_coef_from_rows.argtypes = [ctypes.c_int, I64, P, P, I64, P]
        lib.oracle_compatible_bases.argtypes = [ctypes.c_int, I64, P]
        lib.oracle_compatible_bases.restype = I64
        lib.oracle_accumulate_pairs.argtypes = [ctypes.c_int, P, P, P, I64, P, P, P, I64, P]
        lib.oracle_coef_from_acc.argtypes = [ctypes.c_int, P, P, I64, P]
        lib.oracle_coefs_freq.argtypes = [ctypes.c_int, P, P, I64, P]
        lib.oracle_povm_coefs.argtypes = [ctypes.c_int, P, P, P, I64, P]
        lib.oracle_povm_coefs_freq.argtypes = [ctypes.c_int, P, P, P, I64, P]
        lib.oracle_povm_coefs_direct.argtypes = [ctypes.c_int, P, P, P, I64, P, P]
        lib.oracle_rho_entries.argtypes = [ctypes.c_int, P, P, P, I64, P]
        lib.oracle_lre.argtypes = [ctypes.c_int, P, ctypes.c_uint64, P, P, P]
        lib.oracle_op_count_step1.restype = ctypes.c_uint64
        lib.oracle_op_count_step2.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(st):
    if st != 0:
        raise OracleError(STATUS.get(st, f"status {st}"))


def _counts(n, counts):
    c = np.ascontiguousarray(counts, dtype=np.uint16)
    if c.shape != (3 ** n, 2 ** n):
        raise ValueError(f"counts must have shape (3^n, 2^n) = {(3 ** n, 2 ** n)}, got {c.shape}")
    return c


def _idx(idx):
    return None if idx is None else np.ascontiguousarray(idx, dtype=np.int64)


def one_qubit_tables():
    """(gamma[6,4], xtx[4,4]): the one-qubit Gamma vectors of projectors X+,X-,Y+,Y-,Z+,Z-
    (eq. 2 with eq. 5 at n = 1) and X^T X (Sec. III)."""
    lib = _load()
    g = np.zeros((6, 4))
    x = np.zeros((4, 4))
    _check(lib.oracle_one_qubit_tables(_ptr(g), _ptr(x)))
    return g, x


def pauli_sums(n, counts, idx=None):
    """Integer numerators T_i = sum_{b,s} c[b][s] prod_k g(a_k,b_k,s_k) (int64)."""
    lib = _load()
    c = _counts(n, counts)
    ix = _idx(idx)
    out = np.zeros(4 ** n if ix is None else len(ix), dtype=np.int64)
    _check(lib.oracle_pauli_sums(n, _ptr(c), _ptr(ix), 0 if ix is None else len(ix), _ptr(out)))
    return out


def basis_sums(n, counts, bases, coefs):
    """Signed sum of basis row b against a compatible coefficient i, per (b, i) pair."""
    lib = _load()
    c = _counts(n, counts)
    b = np.ascontiguousarray(bases, dtype=np.int64)
    i = np.ascontiguousarray(coefs, dtype=np.int64)
    out = np.zeros(len(b), dtype=np.int64)
    _check(lib.oracle_basis_sums(n, _ptr(c), _ptr(b), _ptr(i), len(b), _ptr(out)))
    return out


def coefs(n, counts, shots=0, n_per_basis=None, idx=None):
    """Pauli expectations e_i = 2^{n/2} theta_i of eq. (3).  shots > 0: uniform shots;
    shots == 0: per-basis totals (n_per_basis, or the row sums when None)."""
    lib = _load()
    c = _counts(n, counts)
    nb = None if n_per_basis is None else np.ascontiguousarray(n_per_basis, dtype=np.uint32)
    ix = _idx(idx)
    out = np.zeros(4 ** n if ix is None else len(ix))
    _check(lib.oracle_coefs(n, _ptr(c), int(shots), _ptr(nb), _ptr(ix),
                            0 if ix is None else len(ix), _ptr(out)))
    return out


def compatible_bases(n, i):
    """Indices of the bases whose Gamma vectors are nonzero at coefficient i (increasing)."""
    lib = _load()
    m = lib.oracle_compatible_bases(n, int(i), None)
    out = np.zeros(m, dtype=np.int64)
    lib.oracle_compatible_bases(n, int(i), _ptr(out))
    return out


def coef_from_rows(n, i, rows, n_per_basis):
    """e_i from the compatible basis rows only (for tensors too large for host memory)."""
    lib = _load()
    r = np.ascontiguousarray(rows, dtype=np.uint16)
    nb = np.ascontiguousarray(n_per_basis, dtype=np.uint32)
    out = np.zeros(1)
    _check(lib.oracle_coef_from_rows(n, int(i), _ptr(r), _ptr(nb), r.shape[0], _ptr(out)))
    return float(out[0])


def accumulate_pairs(n, rows, bases, n_per_basis, pair_row, pair_coef, pair_slot, acc):
    """Streaming eq. (3), per-basis branch: acc[pair_slot[p]] += S(row pair_row[p],
    coefficient pair_coef[p]) / N_b for every pair (acc: numpy longdouble, updated in
    place).  rows: uint16 [nrows, 2^n] of the bases `bases` with totals `n_per_basis`."""
    lib = _load()
    r = np.ascontiguousarray(rows, dtype=np.uint16)
    b = np.ascontiguousarray(bases, dtype=np.int64)
    nb = np.ascontiguousarray(n_per_basis, dtype=np.uint32)
    pr = np.ascontiguousarray(pair_row, dtype=np.int64)
    pc = np.ascontiguousarray(pair_coef, dtype=np.int64)
    ps = np.ascontiguousarray(pair_slot, dtype=np.int64)
    if acc.dtype != np.longdouble or not acc.flags.c_contiguous:
        raise ValueError("acc must be a contiguous numpy longdouble array")
    if r.shape != (len(b), 2 ** n) or len(nb) != len(b) or not (len(pr) == len(pc) == len(ps)):
        raise ValueError("inconsistent row / pair arrays")
    if len(ps) and (ps.min() < 0 or ps.max() >= len(acc)):
        raise ValueError("pair slot outside acc")
    _check(lib.oracle_accumulate_pairs(n, _ptr(r), _ptr(b), _ptr(nb), len(b), _ptr(pr), _ptr(pc), _ptr(ps),
                                       len(ps), _ptr(acc)))


def coef_from_acc(n, coefs, acc):
    """e_i = acc_i / (X^T X)_ii for completed sums (see accumulate_pairs)."""
    lib = _load()
    c = np.ascontiguousarray(coefs, dtype=np.int64)
    a = np.ascontiguousarray(acc, dtype=np.longdouble)
    out = np.zeros(len(c))
    _check(lib.oracle_coef_from_acc(n, _ptr(c), _ptr(a), len(c), _ptr(out)))
    return out


def povm_coefs(n, counts, G, idx=None):
    """Eq. (3) for the reduced set of 4^n product operators with per-qubit Pauli components
    G[j][a] = Tr(E_j sigma_a) (4 x 4, invertible): e_i = 2^{n/2} theta_i from counts[4^n]
    (outcome j = sum_k j_k 4^{n-k}), p = c / sum(c).  n <= 8."""
    lib = _load()
    c = np.ascontiguousarray(counts, dtype=np.uint16).ravel()
    if c.size != 4 ** n:
        raise ValueError("counts must hold 4^n outcomes")
    g = np.ascontiguousarray(G, dtype=np.float64).reshape(4, 4)
    ix = _idx(idx)
    out = np.zeros(4 ** n if ix is None else len(ix))
    _check(lib.oracle_povm_coefs(n, _ptr(c), _ptr(g), _ptr(ix), 0 if ix is None else len(ix), _ptr(out)))
    return out


def povm_coefs_direct(n, counts, G, idx):
    """Selected coefficients of povm_coefs, each from the O(n 4^n) entrywise product of
    the Kronecker-structured (X^T X)^{-1} row and Gamma^(j) (any n); also returns the
    scale 2^n sum_j p_j prod_k |w[a_k][j_k]| of each coefficient's terms."""
    lib = _load()
    c = np.ascontiguousarray(counts, dtype=np.uint16).ravel()
    if c.size != 4 ** n:
        raise ValueError("counts must hold 4^n outcomes")
    g = np.ascontiguousarray(G, dtype=np.float64).reshape(4, 4)
    ix = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.zeros(len(ix))
    cond = np.zeros(len(ix))
    _check(lib.oracle_povm_coefs_direct(n, _ptr(c), _ptr(g), _ptr(ix), len(ix), _ptr(out), _ptr(cond)))
    return out, cond


def povm_coefs_freq(n, freq, G, idx=None):
    """povm_coefs with given frequencies p[4^n] (float64)."""
    lib = _load()
    f = np.ascontiguousarray(freq, dtype=np.float64).ravel()
    if f.size != 4 ** n:
        raise ValueError("freq must hold 4^n outcomes")
    g = np.ascontiguousarray(G, dtype=np.float64).reshape(4, 4)
    ix = _idx(idx)
    out = np.zeros(4 ** n if ix is None else len(ix))
    _check(lib.oracle_povm_coefs_freq(n, _ptr(f), _ptr(g), _ptr(ix), 0 if ix is None else len(ix), _ptr(out)))
    return out


def coefs_freq(n, freq, idx=None):
    """Eq. (3) evaluated on given frequencies p[b][s] (float64, shape (3^n, 2^n))."""
    lib = _load()
    f = np.ascontiguousarray(freq, dtype=np.float64)
    if f.shape != (3 ** n, 2 ** n):
        raise ValueError("freq must have shape (3^n, 2^n)")
    ix = _idx(idx)
    out = np.zeros(4 ** n if ix is None else len(ix))
    _check(lib.oracle_coefs_freq(n, _ptr(f), _ptr(ix), 0 if ix is None else len(ix), _ptr(out)))
    return out


def rho(n, coef, rows=None, cols=None):
    """Eq. (4): mu = 2^{-n} sum_i e_i (x)_k sigma_{a_k}.  All entries (complex128, shape
    (2^n, 2^n)) or the listed (row, col) entries."""
    lib = _load()
    e = np.ascontiguousarray(coef, dtype=np.float64)
    if e.shape != (4 ** n,):
        raise ValueError("coef must have length 4^n")
    if rows is None:
        out = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
        _check(lib.oracle_rho_entries(n, _ptr(e), None, None, 0, _ptr(out)))
        return out
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(len(r), dtype=np.complex128)
    _check(lib.oracle_rho_entries(n, _ptr(e), _ptr(r), _ptr(c), len(r), _ptr(out)))
    return out


def lre(n, counts, shots=0, n_per_basis=None):
    """Whole path on one instance: (coef[4^n], rho[2^n, 2^n])."""
    e = coefs(n, counts, shots, n_per_basis)
    return e, rho(n, e)


def reset_op_counts():
    _load().oracle_reset_op_counts()


def op_counts():
    lib = _load()
    return int(lib.oracle_op_count_step1()), int(lib.oracle_op_count_step2())
