"""Expected values for the 14-qubit Philox workload (per-basis totals), computed by the
CPU oracle alone.

The count tensor (3^14 bases x 2^14 outcomes, 156.7 GB) does not fit host memory, so
the oracle streams it: every basis row it needs is regenerated with the CPU Philox twin
(tomo_inputs, input generation only) and eq. (3) is accumulated over the (basis,
coefficient) pairs that are not identically zero (oracle.accumulate_pairs, the paper's
own per-group sum of Sec. III), then divided by (X^T X)_ii (Sec. III).  Entries of mu
follow from eq. (4) on those coefficients (oracle.rho).

Coefficients (all computed):
  * i = 0 (all 3^14 bases), 6 of weight 1 (3^13 bases each), 20 of weight 2 (3^12 each),
    20 of weight 3 and 20 of weight 4;
  * 10^4 uniform on [1, 4^14);
  * for 5 nonzero patterns x (x_k = 1 where qubit k is off-diagonal; popcounts 14, 13,
    12, 11, 10), all 2^14 coefficients with letters in {X, Y} where x_k = 1 and {I, Z}
    where x_k = 0 -- exactly the coefficients entering mu[r][r ^ x] (Sec. IV groups);
    400 of each pattern are stored as coefficient checks.
mu: 2000 rows r per pattern, entries (r, r ^ x): 10^4 entries.

Run from the repository root (about 20 minutes on 8 cores):
    python tests/golden/make_n14_spotchecks.py
writes tests/golden/n14_spotchecks.npz.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import tomo_inputs as ti  # noqa: E402

N = 14
SEED14 = 0x16020860414
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "n14_spotchecks.npz")


def index_of(letters):
    """Pauli index from letters by position p (p = 0 least significant, qubit n - p)."""
    return int(sum(int(a) << (2 * p) for p, a in enumerate(letters)))


def pattern_coefs(x):
    """All 2^n coefficients entering mu[r][r ^ x]: letter X/Y where bit p of x is set,
    I/Z where it is clear (z selects the second letter of each pair)."""
    z = np.arange(1 << N, dtype=np.int64)
    i = np.zeros(1 << N, dtype=np.int64)
    for p in range(N):
        xb = (x >> p) & 1
        zb = (z >> p) & 1
        letter = np.where(xb == 1, np.where(zb == 1, 2, 1), np.where(zb == 1, 3, 0))
        i |= letter.astype(np.int64) << (2 * p)
    return i


def main():
    rng = np.random.default_rng(1414)
    groups = {}
    groups["trace"] = np.array([0], dtype=np.int64)
    w1 = set()
    while len(w1) < 6:
        letters = [0] * N
        letters[int(rng.integers(0, N))] = int(rng.integers(1, 4))
        w1.add(index_of(letters))
    groups["weight1"] = np.array(sorted(w1), dtype=np.int64)
    w2 = set()
    while len(w2) < 20:
        p1, p2 = rng.choice(N, size=2, replace=False)
        letters = [0] * N
        letters[p1], letters[p2] = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        w2.add(index_of(letters))
    groups["weight2"] = np.array(sorted(w2), dtype=np.int64)
    for w in (3, 4):                       # 3^11 and 3^10 compatible bases each
        ws = set()
        while len(ws) < 20:
            pos = rng.choice(N, size=w, replace=False)
            letters = [0] * N
            for p in pos:
                letters[p] = int(rng.integers(1, 4))
            ws.add(index_of(letters))
        groups[f"weight{w}"] = np.array(sorted(ws), dtype=np.int64)
    groups["uniform"] = rng.integers(1, 4 ** N, size=10_000, dtype=np.int64)
    patterns = []
    for pc in (14, 13, 12, 11, 10):
        bits = rng.choice(N, size=pc, replace=False)
        patterns.append(int(sum(1 << int(b) for b in bits)))
    pat_coefs = [pattern_coefs(x) for x in patterns]

    # every coefficient to evaluate, once
    wanted = np.unique(np.concatenate(list(groups.values()) + pat_coefs))
    print(f"{len(wanted)} coefficients", flush=True)

    # (basis, coefficient) pairs that are not identically zero, sorted by basis (stable:
    # each coefficient's bases stay in increasing order, as in oracle.coef_from_rows)
    t0 = time.time()
    pb, ps = [], []
    for t, i in enumerate(wanted):
        b = oracle.compatible_bases(N, int(i))
        pb.append(b)
        ps.append(np.full(len(b), t, dtype=np.int64))
    pb = np.concatenate(pb)
    ps = np.concatenate(ps)
    order = np.argsort(pb, kind="stable")
    pb, ps = pb[order], ps[order]
    pc = wanted[ps]
    del order
    print(f"{len(pb)} pairs in {time.time() - t0:.0f} s", flush=True)

    acc = np.zeros(len(wanted), dtype=np.longdouble)
    ubases = np.unique(pb)
    chunk = 4096
    t0 = time.time()
    lo = 0
    for c0 in range(0, len(ubases), chunk):
        bases = ubases[c0:c0 + chunk]
        rows, nb = ti.philox_counts_rows_fast(N, SEED14, bases)      # input generation
        hi = np.searchsorted(pb, bases[-1], side="right")
        prow = np.searchsorted(bases, pb[lo:hi])
        oracle.accumulate_pairs(N, rows, bases, nb, prow, pc[lo:hi], ps[lo:hi], acc)
        lo = hi
        if (c0 // chunk) % 100 == 0:
            el = time.time() - t0
            print(f"  bases {c0 + len(bases)}/{len(ubases)}  {el:.0f} s", flush=True)
    assert lo == len(pb)
    e = oracle.coef_from_acc(N, wanted, acc)
    val = dict(zip(wanted.tolist(), e.tolist()))

    coef_idx, coef_val, coef_group = [], [], []
    names = list(groups) + ["pattern"]
    for g, idx in groups.items():
        coef_idx.append(idx)
        coef_group.append(np.full(len(idx), names.index(g), dtype=np.int8))
    for k, pcs in enumerate(pat_coefs):
        pick = rng.choice(len(pcs), size=400, replace=False)
        coef_idx.append(pcs[pick])
        coef_group.append(np.full(400, names.index("pattern"), dtype=np.int8))
    coef_idx = np.concatenate(coef_idx)
    coef_val = np.array([val[int(i)] for i in coef_idx])
    coef_group = np.concatenate(coef_group)

    # eq. (4) on the oracle's coefficients; every other coefficient is NaN, so an entry
    # that needed one outside the computed patterns would come out NaN
    full = np.full(4 ** N, np.nan)
    full[wanted] = e
    rr, pid = [], []
    for k, x in enumerate(patterns):
        r = rng.integers(0, 1 << N, size=2000, dtype=np.int64)
        rr.append(r)
        pid.append(np.full(2000, k, dtype=np.int8))
    rr = np.concatenate(rr)
    pid = np.concatenate(pid)
    cc = rr ^ np.array(patterns, dtype=np.int64)[pid]
    mu = oracle.rho(N, full, rr, cc)
    del full
    assert np.all(np.isfinite(mu.real)) and np.all(np.isfinite(mu.imag))

    np.savez_compressed(OUT, n=N, seed=np.uint64(SEED14), group_names=np.array(names),
                        coef_idx=coef_idx, coef_val=coef_val, coef_group=coef_group,
                        patterns=np.array(patterns, dtype=np.int64), rho_row=rr.astype(np.int32),
                        rho_pattern=pid, rho_val=mu)
    print(f"wrote {OUT}: {len(coef_idx)} coefficients, {len(rr)} mu entries", flush=True)


if __name__ == "__main__":
    main()
