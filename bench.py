#!/usr/bin/env python3
"""Benchmark of the LRE hot path (steps (i) + (ii)) on one MI355X.

Default workload: n = 14 qubits, 3^14 = 4,782,969 Pauli bases x 2^14 outcomes of
uint16 counts (156.7 GB, resident in HBM before timing), generated on the device
from Philox4x32-10 (i.i.d. uniform on {0..12}) with per-basis totals N_b; outputs
the 4^14 binary64 Pauli coefficients and the 16384 x 16384 complex128 matrix mu.
One step = one lre_estimate call (every kernel of steps (i) and (ii)).

Prints ONE JSON line with throughput (counts/s over the whole step), the roofline of
the dominant kernel (the counts pass) measured live with HIP events on the stream it
runs on, and the CPU oracle timed on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload n14|n12|n8|batch|project|stream15|povm14]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "counts/sec + end-to-end LRE time at n=12,14; int8-MFMA vs plain, exact sums"
HBM_PEAK_GBS = 8000.0
SEED14 = 0x16020860414


def _hip():
    lib = ctypes.CDLL("libamdhip64.so")
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    lib.hipEventSynchronize.argtypes = [ctypes.c_void_p]
    return lib


class StageEvents:
    """4 HIP events per timed step, recorded by the library at stage boundaries."""

    def __init__(self, steps):
        self.hip = _hip()
        self.ev = []
        for _ in range(steps):
            row = []
            for _ in range(4):
                e = ctypes.c_void_p()
                if self.hip.hipEventCreate(ctypes.byref(e)) != 0:
                    raise RuntimeError("hipEventCreate failed")
                row.append(e.value)
            self.ev.append(row)

    def ms(self, step, a, b):
        out = ctypes.c_float()
        self.hip.hipEventSynchronize(ctypes.c_void_p(self.ev[step][b]))
        rc = self.hip.hipEventElapsedTime(ctypes.byref(out), ctypes.c_void_p(self.ev[step][a]),
                                          ctypes.c_void_p(self.ev[step][b]))
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({rc})")
        return float(out.value)

    def close(self):
        for row in self.ev:
            for e in row:
                self.hip.hipEventDestroy(ctypes.c_void_p(e))


def measured_traffic(workload, tiles=None):
    """HBM bytes per launch of the workload's dominant kernel (the counts pass; the batch
    kernel for the batch) from the committed rocprofv3 PMC summary, if it was taken on the
    current kernel source (and, for the batch, with the same work-item shape `tiles`);
    else None."""
    name = "batch_kernel_512_instances" if workload == "batch" else f"fold_counts_{workload}"
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    from paper_1602_08604_amd.profsum import kernel_source_hash
    if rec.get("kernel_source_hash") != kernel_source_hash(workload):
        return None
    if tiles is not None and f"--batch-tiles {tiles} " not in rec.get("command_fetch", ""):
        return None
    return rec.get("hbm_bytes_per_launch")


def make_workload(name, torch):
    import tomo_inputs.gpu as tg
    dev = "cuda:0"
    if name == "n14":
        n = 14
        counts, nb = tg.philox_counts(n, SEED14, device=dev)
        desc = ("n=14: 4782969 bases x 16384 outcomes uint16 (156.7 GB in HBM), Philox4x32-10 "
                "i.i.d. U{0..12}, per-basis totals N_b; coef f64 [4^14] + rho c128 [16384^2]")
        return n, counts, 0, nb, desc
    if name == "n12":
        n = 12
        counts = tg.ghz_multinomial_counts(n, 0.05, 10_000, seed=16021, device=dev)
        desc = ("n=12: 531441 bases x 4096 outcomes uint16 (4.35 GB in HBM), GHZ_12 with "
                "depolarising p=0.05, multinomial 10^4 shots/basis; coef f64 [4^12] + rho c128 [4096^2]")
        return n, counts, 10_000, None, desc
    if name == "n8":
        import numpy as np
        import tomo_inputs as ti
        n = 8
        rng = np.random.default_rng(16041)
        G = ti.ginibre_factor(n, 4, rng)
        c = ti.multinomial_counts(ti.born_probs_mixed(n, G), 10_000, rng)
        desc = ("n=8: 6561 bases x 256 outcomes uint16, rank-4 Ginibre state, multinomial 10^4 "
                "shots/basis; coef f64 [4^8] + rho c128 [256^2]")
        return n, torch.from_numpy(c).to(dev), 10_000, None, desc
    raise SystemExit(f"unknown workload {name}")


FP64_PEAK_TFS = 78.6


def bench_project(args, torch, lre):
    """Step (iii) (lre_project) at n = --project-n: mu from 200-shot counts of a Haar pure
    state (n <= 12) or from the Philox per-basis workload (n = 13, 14), so that many
    eigenvalues are truncated.  The flop count is the usual one of a complex Hermitian
    eigendecomposition with eigenvectors (reduction to tridiagonal form 16/3 d^3,
    tridiagonal divide and conquer ~4/3 d^3, back-transformation 8 d^3 real flops) plus
    the reassembly product (8 d^3); the step is dense FP64 library work."""
    import tomo_inputs.gpu as tg
    n = args.project_n
    d = 1 << n
    if n <= 12:
        shots = 200
        counts = tg.haar_multinomial_counts(n, shots, 16043, device="cuda:0")
        _, mu = lre.estimate(counts, shots)
        src = f"mu from {shots}-shot multinomial counts of a Haar pure state"
    else:
        counts, nb = tg.philox_counts(n, SEED14 if n == 14 else SEED14 + 1, device="cuda:0")
        _, mu = lre.estimate(counts, 0, n_per_basis=nb)
        del nb
        src = "mu from the Philox per-basis workload (i.i.d. U{0..12} counts)"
    del counts
    torch.cuda.empty_cache()
    rho = torch.empty_like(mu)
    ev = torch.empty(d, dtype=torch.float64, device="cuda:0")
    ws = torch.empty(lre.lib().lre_project_workspace_bytes(n), dtype=torch.uint8, device="cuda:0")
    for _ in range(max(1, args.warmup)):
        lre.project(mu, rho, ev, ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        lre.project(mu, rho, ev, ws, check=False)
    e1.record()
    torch.cuda.synchronize()
    lre.check_flags("cuda:0")
    ms = e0.elapsed_time(e1) / args.steps
    flops = (16.0 / 3 + 4.0 / 3 + 8.0 + 8.0) * float(d) ** 3
    kept = int((ev > 0).sum().item())
    out = {
        "metric": "step (iii) time (closest physical state)", "value": ms, "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"n={n}: {src}; complex128 [{d}^2]; {kept} of {d} eigenvalues of mu positive",
                   "n": n},
        "roofline": {"bound": "mfma", "achieved": flops / (ms / 1e3) / 1e12, "peak": FP64_PEAK_TFS,
                     "unit": "TFLOP/s", "frac": flops / (ms / 1e3) / 1e12 / FP64_PEAK_TFS, "traffic": None,
                     "kernel": "rocsolver_zheevd + spectrum kernel + rocblas_zgemm",
                     "algorithmic_flops_per_step": flops},
    }
    print(f"[bench] project n={n}: {ms:.3f} ms/step, {kept} of {d} eigenvalues positive", file=sys.stderr,
          flush=True)
    print(json.dumps(out), flush=True)


def measured_hbm(torch, lre, gib=8, reps=5):
    """Practical HBM rates of this device next to the 8 TB/s datasheet peak: the library's
    streaming read (lre_stream_read) and copy (lre_stream_copy, read + write) over `gib`
    GiB, timed with events on the current stream after one warm-up each."""
    n = gib << 28
    x = torch.ones(n, dtype=torch.int32, device="cuda:0")
    y = torch.empty_like(x)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    nbytes = 4.0 * n

    def rate(fn, moved):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return moved * reps / (e0.elapsed_time(e1) / 1e3) / 1e9

    read = rate(lambda: lre.stream_read(x, sink), nbytes)
    copy = rate(lambda: lre.stream_copy(x, y), 2.0 * nbytes)
    del x, y, sink
    torch.cuda.empty_cache()
    return {"stream_read_gbs": read, "stream_copy_gbs": copy, "unit": "GB/s", "bytes_each": nbytes,
            "how": f"lre_stream_read / lre_stream_copy (16-byte nontemporal vectors, a contiguous range per block) over {gib} GiB, "
                   f"{reps} reps each; copy counts read + write bytes"}


def measured_compute(torch, lre, reps=5):
    """Issue rates of the two compute paths next to their datasheet peaks: 32-bit
    integer adds (lre_peak_valu_i32) and dense int8 MFMA (lre_peak_mfma_i8), each timed
    with events over `reps` launches after one warm-up."""
    sink = torch.zeros(1, dtype=torch.int32, device="cuda:0")

    def rate(kind, iters):
        lre.peak_rate(kind, iters, sink)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ops = 0.0
        for _ in range(reps):
            ops += lre.peak_rate(kind, iters, sink)
        e1.record()
        torch.cuda.synchronize()
        return ops / (e0.elapsed_time(e1) / 1e3) / 1e12

    valu = rate("valu_i32", 2000)
    mfma = rate("mfma_i8", 20000)
    return {"valu_int32_tops": valu, "valu_int32_datasheet_tops": 78.6, "mfma_int8_tops": mfma,
            "mfma_int8_datasheet_tops": 5000.0, "unit": "Tops",
            "how": "lre_peak_valu_i32 (8 independent add chains per lane) and lre_peak_mfma_i8 "
                   "(4 independent v_mfma_i32_16x16x64_i8 chains per wave), 8 workgroups of 256 per CU, "
                   f"{reps} launches each"}


def host_cpu():
    """Model name and logical CPU count of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def _omp_set_threads(k):
    """Thread count of the oracle's OpenMP loops (libgomp, shared by the process)."""
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))
    except OSError:
        pass


def _n14_pairs_rate(n, rng, budget_s, threads):
    """Oracle rate on the 14-qubit workload: coefficients with <= 4 identity letters (at
    most 81 compatible bases each) in chunks of 48; their rows are regenerated by the C
    Philox twin (input generation, not timed) and eq. (3) accumulated over the pairs by
    oracle.accumulate_pairs (OpenMP over pairs) with `threads` threads.  Returns
    (visited terms per second, coefficients, seconds)."""
    import numpy as np

    import oracle
    import tomo_inputs as ti
    _omp_set_threads(threads)
    t_acc, visits, ncoef = 0.0, 0, 0
    while t_acc < budget_s:
        coefs, bases_all = [], []
        for _ in range(48):
            letters = rng.integers(1, 4, size=n)
            letters[rng.choice(n, size=int(rng.integers(0, 5)), replace=False)] = 0
            i = int(sum(int(a) * 4 ** (n - 1 - k) for k, a in enumerate(letters)))
            coefs.append(i)
            bases_all.append(oracle.compatible_bases(n, i))
        ub = np.unique(np.concatenate(bases_all))
        rows, nb = ti.philox_counts_rows_fast(n, SEED14, ub)             # input generation
        prow = np.concatenate([np.searchsorted(ub, b) for b in bases_all])
        pcoef = np.concatenate([np.full(len(b), i, dtype=np.int64) for i, b in zip(coefs, bases_all)])
        pslot = np.concatenate([np.full(len(b), t, dtype=np.int64) for t, b in enumerate(bases_all)])
        acc = np.zeros(len(coefs), dtype=np.longdouble)
        t0 = time.perf_counter()
        oracle.accumulate_pairs(n, rows, ub, nb, prow, pcoef, pslot, acc)
        oracle.coef_from_acc(n, np.array(coefs, dtype=np.int64), acc)
        t_acc += time.perf_counter() - t0
        visits += len(prow) * 2 ** n
        ncoef += len(coefs)
    return visits / t_acc, ncoef, t_acc


def cpu_baseline(workload, n, shots, counts_dev, coef_dev, budget_s=12.0):
    """Time the CPU oracle (as it stands) on a bounded sample of the same workload and
    extrapolate to the whole step: step (i) visits 12^n (projector, coefficient) terms,
    step (ii) 8^n (coefficient, entry) terms."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(7)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count()))
    if workload == "n14":
        # all of the host's threads, then one thread (the step-(ii) terms cost the same
        # per visit as the step-(i) ones: one multiply-add over a row or an entry's terms)
        rate_all, nc_all, t_all = _n14_pairs_rate(n, rng, budget_s * 0.5, cores)
        rate_one, nc_one, t_one = _n14_pairs_rate(n, rng, budget_s * 0.5, 1)
        _omp_set_threads(cores)
        terms = 12.0 ** n + 8.0 ** n
        full_all, full_one = terms / rate_all, terms / rate_one
        sample = (f"{nc_all} coefficients (<= 81 bases each, rows regenerated by the C Philox twin) "
                  f"in {t_all:.1f} s on {cores} threads; extrapolated to the whole step "
                  f"({full_all / 3600:.3g} h for 12^n + 8^n terms)")
        return {"value": 6.0 ** n / full_all, "unit": "counts/s", "cores": cores, "kind": "oracle",
                "host": host_cpu(), "sample": sample,
                "one_core": {"value": 6.0 ** n / full_one, "unit": "counts/s", "cores": 1,
                             "sample": f"{nc_one} coefficients in {t_one:.1f} s on 1 thread "
                                       f"({full_one / 3600:.3g} h extrapolated)"}}
    visits_i = 0
    t_i = 0.0
    ncoef = 0
    c = counts_dev.cpu().numpy()
    # batches of 4096 random coefficients until about 3/4 of the budget is spent
    while t_i < budget_s * 0.75:
        idx = rng.integers(0, 4 ** n, size=4096)
        w = np.array([sum(1 for k in range(n) if (int(j) >> (2 * k)) & 3) for j in idx])
        t0 = time.perf_counter()
        oracle.coefs(n, c, shots, idx=idx)
        t_i += time.perf_counter() - t0
        visits_i += int(np.sum(3.0 ** (n - w))) * 2 ** n
        ncoef += len(idx)
    sample = f"{ncoef} random coefficients of the full count tensor"
    # step (ii): sampled entries of eq. (4) on the GPU coefficients
    coef = coef_dev.cpu().numpy()
    r = rng.integers(0, 2 ** n, 2000)
    cc = rng.integers(0, 2 ** n, 2000)
    t0 = time.perf_counter()
    oracle.rho(n, coef, r, cc)
    t_ii = time.perf_counter() - t0
    visits_ii = 2000 * 2 ** n
    t_full = 12.0 ** n / (visits_i / t_i) + 8.0 ** n / (visits_ii / t_ii)
    return {"value": 6.0 ** n / t_full, "unit": "counts/s", "cores": cores, "kind": "oracle", "host": host_cpu(),
            "sample": f"{sample}; oracle time {t_i + t_ii:.1f} s, extrapolated to the whole "
                      f"step ({t_full / 3600:.3g} h for 12^n + 8^n terms)"}


SEED15 = 0x16020860415


def bench_stream(args, torch, lre):
    """Streamed estimate at n = 15 (940 GB of counts, beyond device memory): 27 slabs of
    3^12 bases (34.8 GB each) of the Philox per-basis workload, each generated on the device
    into one slab buffer (not timed) and pushed (timed with events around every push and
    the finish).  Then the host path at n = 14 (27 slabs of 5.8 GB): each slab copied from
    pinned host memory by lre_stream_push_host, against the measured host-to-device rate."""
    import tomo_inputs.gpu as tg
    n, h = 15, 3
    rows = 3 ** (n - h)
    S = lre.Stream(n, h, 0)
    S.workspace()
    slab = torch.empty((rows, 2 ** n), dtype=torch.uint16, device="cuda:0")
    nb = torch.empty(rows, dtype=torch.int32, device="cuda:0")
    coef = torch.empty(4 ** n, dtype=torch.float64, device="cuda:0")
    rho = torch.empty((2 ** n, 2 ** n), dtype=torch.complex128, device="cuda:0")
    t_push = 0.0
    S.begin(coef)
    for k in range(3 ** h):
        tg.philox_counts(n, SEED15, b_begin=k * rows, b_count=rows, counts=slab, nb=nb)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        S.push(k, slab, nb)
        e1.record()
        torch.cuda.synchronize()
        t_push += e0.elapsed_time(e1)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    S.finish(rho, check=False)
    e1.record()
    torch.cuda.synchronize()
    lre.check_flags("cuda:0")
    t_fin = e0.elapsed_time(e1)
    S.close()
    del slab, nb, coef, rho
    torch.cuda.empty_cache()
    ms = t_push + t_fin
    n_counts = 3 ** n * 2 ** n
    algo = 2.0 * n_counts + 24.0 * 4 ** n
    slab_counts = rows * 2 ** n
    achieved = 2.0 * slab_counts / (t_push / 3 ** h / 1e3) / 1e9   # per push: every pass of the slab
    print(f"[bench] stream n=15: {3 ** h} slabs pushed in {t_push:.1f} ms, finish {t_fin:.1f} ms", file=sys.stderr,
          flush=True)

    # host path (n = 14): slabs in pinned host memory
    n2 = 14
    rows2 = 3 ** (n2 - h)
    host = torch.empty((rows2, 2 ** n2), dtype=torch.uint16, pin_memory=True)
    dev = torch.empty((rows2, 2 ** n2), dtype=torch.uint16, device="cuda:0")
    nbh = torch.empty(rows2, dtype=torch.int32, pin_memory=True)
    nbd = torch.empty(rows2, dtype=torch.int32, device="cuda:0")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    host.copy_(dev)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(3):
        dev.copy_(host, non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    h2d = 3 * 2.0 * rows2 * 2 ** n2 / (e0.elapsed_time(e1) / 1e3) / 1e9
    S2 = lre.Stream(n2, h, 0, flags=lre.LRE_STREAM_HOST)
    S2.workspace()
    coef2 = torch.empty(4 ** n2, dtype=torch.float64, device="cuda:0")
    rho2 = torch.empty((2 ** n2, 2 ** n2), dtype=torch.complex128, device="cuda:0")
    S2.begin(coef2)
    t_host = 0.0
    for k in range(3 ** h):
        tg.philox_counts(n2, SEED14, b_begin=k * rows2, b_count=rows2, counts=dev, nb=nbd)
        host.copy_(dev)
        nbh.copy_(nbd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S2.push_host(k, host, nbh)
        torch.cuda.synchronize()
        t_host += time.perf_counter() - t0
    t0 = time.perf_counter()
    S2.finish(rho2)
    t_host += time.perf_counter() - t0
    S2.close()
    host_rate = 3 ** n2 * 2 ** n2 / t_host
    out = {
        "metric": METRIC + " (streamed, n = 15)", "value": n_counts / (ms / 1e3), "unit": "counts/s",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32+f64", "data": "synthetic",
        "config": {"workload": "n=15: 14348907 bases x 32768 outcomes uint16 (940 GB, more than device memory), "
                               "Philox4x32-10 i.i.d. U{0..12}, per-basis totals; 27 device slabs of 3^12 bases "
                               "(34.8 GB) generated one at a time (generation not timed) and pushed; coef f64 "
                               "[4^15] + rho c128 [32768^2]", "n": 15, "h": h, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "one slab push (totals, the 8 segments' counts and later passes, row check, "
                               "top-qubit fold), timed with events around each push",
                     "algorithmic_bytes_per_launch": 2.0 * slab_counts},
        "whole_step_hbm_frac": algo / (ms / 1e3) / (HBM_PEAK_GBS * 1e9),
        "step_ms": {"pushes": t_push, "finish": t_fin},
        "host_streamed_n14": {"counts_per_s": host_rate, "s": t_host, "h2d_pinned_gbs": h2d,
                              "link_bound_counts_per_s": h2d * 1e9 / 2.0,
                              "how": "27 slabs of 3^11 bases (5.8 GB) copied from pinned host memory by "
                                     "lre_stream_push_host, wall time of the pushes and the finish"},
    }
    print(json.dumps(out), flush=True)


def bench_povm(args, torch, lre):
    """Reduced operator set (Sec. VI) at n = 14: 4^14 outcome counts of the tetrahedral POVM
    (uniform random counts in [0, 60), seeded), coefficients and rho."""
    import numpy as np
    n = 14
    rng = np.random.default_rng(16044)
    c = torch.from_numpy(rng.integers(0, 60, size=4 ** n).astype(np.uint16)).to("cuda:0")
    tet = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]]) / np.sqrt(3.0)
    G = torch.from_numpy(np.hstack([np.full((4, 1), 0.5), tet / 2])).to("cuda:0")
    d = 1 << n
    coef = torch.empty(4 ** n, dtype=torch.float64, device="cuda:0")
    rho = torch.empty((d, d), dtype=torch.complex128, device="cuda:0")
    ws = torch.empty(lre.lib().lre_povm_workspace_bytes(n, 0), dtype=torch.uint8, device="cuda:0")
    for _ in range(args.warmup):
        lre.povm_estimate(c, G, coef=coef, rho=rho, workspace=ws, check=False)
    lre.check_flags("cuda:0")
    ev = StageEvents(args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        lre.set_stage_events(ev.ev[k])
        lre.povm_estimate(c, G, coef=coef, rho=rho, workspace=ws, check=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lre.set_stage_events(None)
    lre.check_flags("cuda:0")
    ms = (t1 - t0) * 1e3 / args.steps
    t_i = sum(ev.ms(k, 1, 2) for k in range(args.steps)) / args.steps
    t_ii = sum(ev.ms(k, 2, 3) for k in range(args.steps)) / args.steps
    ev.close()
    m = 4 ** n
    algo_i = 2.0 * m + 8.0 * m
    out = {
        "metric": "reduced operator set (Sec. VI): outcomes/s of LRE steps (i) + (ii)", "value": m / (ms / 1e3),
        "unit": "counts/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "n=14: 4^14 outcome counts uint16 (537 MB) of the tetrahedral POVM on every qubit, "
                               "uniform random in [0, 60); coef f64 [4^14] + rho c128 [16384^2]", "n": n,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": algo_i / (t_i / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": algo_i / (t_i / 1e3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "step (i) mode-product passes (povm_low_kernel, povm_high4_kernel x2)",
                     "algorithmic_bytes_per_launch": algo_i},
        "step_ms": {"step_i": t_i, "step_ii": t_ii},
        "whole_step_hbm_frac": (algo_i + 16.0 * m) / (ms / 1e3) / (HBM_PEAK_GBS * 1e9),
    }
    print(f"[bench] povm n=14: {ms:.3f} ms/step (step (i) {t_i:.3f} ms, step (ii) {t_ii:.3f} ms)", file=sys.stderr,
          flush=True)
    print(json.dumps(out), flush=True)


BATCH_SEED = 16042


def batch_instances(torch):
    """512 instances: n uniform in {3..9} and shots uniform in [100, 10^4] from
    default_rng(16042); instance j is a Haar pure state with its own seed 16042*1000 + j,
    multinomial counts drawn on the device."""
    import numpy as np
    import tomo_inputs.gpu as tg
    rng = np.random.default_rng(BATCH_SEED)
    ns = [int(x) for x in rng.integers(3, 10, size=512)]
    shots = [int(x) for x in rng.integers(100, 10_001, size=512)]
    counts = [tg.haar_multinomial_counts(n, s, BATCH_SEED * 1000 + j, device="cuda:0")
              for j, (n, s) in enumerate(zip(ns, shots))]
    return ns, shots, counts


def bench_batch(args, torch, lre):
    t0 = time.time()
    ns, shots, counts = batch_instances(torch)
    torch.cuda.synchronize()
    t_gen = time.time() - t0
    bflags = lre.LRE_NO_RHO if args.no_rho else 0
    b = lre.Batch(counts, shots, flags=bflags)
    t0 = time.time()
    if args.batch_tiles:
        # a fixed work-item shape (e.g. the one the tuner chose in an earlier run), so that
        # a profile of this run holds the timed launches only
        b.set_tiles(*[int(v) for v in args.batch_tiles.split(",")])
        tuned_ms = None
    else:
        tuned_ms = b.tune(reps=3)
    t_tune = time.time() - t0
    tiles = b.tiles
    b.run(check=True)
    ws = b.workspace()
    # one captured launch (fill kernel + persistent kernel), replayed per step
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        b.run()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lre.check_flags("cuda:0")
    ms_step = (t1 - t0) * 1e3 / args.steps
    ms_dev = e0.elapsed_time(e1) / args.steps
    n_counts = sum(3 ** n * 2 ** n for n in ns)
    algo = sum(2.0 * 6 ** n + 8.0 * 4 ** n + (0.0 if args.no_rho else 16.0 * 4 ** n) for n in ns)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    # FP32 rho error against FP64 over all instances
    err_abs, err_fro = None, None
    if not args.no_compare and not args.no_rho:
        b32 = lre.Batch(counts, shots, flags=lre.LRE_RHO_FP32)
        b32.run(check=True)
        err_abs, err_fro = 0.0, 0.0
        for r32, r64 in zip(b32.rhos, b.rhos):
            dlt = r32.to(torch.complex128) - r64
            err_abs = max(err_abs, dlt.abs().max().item())
            err_fro = max(err_fro, (torch.linalg.norm(dlt) / torch.linalg.norm(r64)).item())
        b32.close()
    print(f"[bench] batch: generated in {t_gen:.1f} s, tuned in {t_tune:.2f} s -> {tiles}; "
          f"{args.steps} replays: {ms_step:.3f} ms/step wall, {ms_dev:.3f} ms/step device", file=sys.stderr, flush=True)
    from collections import Counter
    hist = dict(sorted(Counter(ns).items()))
    out = {
        "metric": METRIC,
        "value": n_counts / (ms_step / 1e3),
        "unit": "counts/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32+f64", "data": "synthetic",
        "config": {"workload": "batched: 512 instances, n uniform in {3..9} (default_rng(16042)), Haar pure "
                               "states, shots uniform in [100, 10^4], uint16 counts; one captured launch "
                               "(counter fill + persistent kernel) per step"
                               + ("; coefficients only (no rho)" if args.no_rho else ""),
                   "instances": 512, "n_histogram": hist, "total_counts": n_counts, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": 2.0 * n_counts / (ms_dev / 1e3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": 2.0 * n_counts / (ms_dev / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None if args.no_rho else measured_traffic(
                         "batch", ",".join(str(tiles[k]) for k in
                                           ("workers_per_cu", "counts_tiles", "fold_cols", "rho_blocks", "interleave", "staged"))),
                     "kernel": ("batch launch: persistent batch_kernel (counts pass, instances of n <= 7), "
                                "batch_fold_kernel, batch_rho_kernel" if tiles.get("staged") else
                                "batch_kernel (persistent, all stages of all instances)"),
                     "algorithmic_bytes_per_launch": 2.0 * n_counts},
        "whole_step_hbm_frac": algo / (ms_dev / 1e3) / (HBM_PEAK_GBS * 1e9),
        "tiles": tiles, "tune_s": t_tune, "tuned_ms": tuned_ms,
        "rho_fp32_vs_fp64": {"max_abs": err_abs, "max_rel_frobenius": err_fro},
    }
    if not args.no_cpu_baseline:
        import numpy as np
        import oracle
        t_cpu, work, done = 0.0, 0.0, 0
        for j in np.random.default_rng(7).permutation(len(ns)):
            if t_cpu > 12.0:
                break
            c = counts[j].cpu().numpy()
            t0 = time.perf_counter()
            e = oracle.coefs(ns[j], c, shots[j])
            oracle.rho(ns[j], e)
            t_cpu += time.perf_counter() - t0
            work += 12.0 ** ns[j] + 8.0 ** ns[j]
            done += 1
        rate = work / t_cpu
        t_full = sum(12.0 ** n + 8.0 ** n for n in ns) / rate
        out["cpu_baseline"] = {"value": n_counts / t_full, "unit": "counts/s",
                               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count())), "kind": "oracle",
                               "host": host_cpu(),
                               "sample": f"full oracle (coef + rho) on {done} randomly chosen instances "
                                         f"({t_cpu:.1f} s), extrapolated by 12^n + 8^n terms to all 512 "
                                         f"({t_full:.0f} s)"}
    b.close()
    out["hbm_measured"] = measured_hbm(torch, lre)
    out["compute_measured"] = measured_compute(torch, lre)
    out["roofline"]["frac_of_measured_read"] = out["roofline"]["achieved"] / out["hbm_measured"]["stream_read_gbs"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="n14", choices=["n14", "n12", "n8", "batch", "project", "stream15", "povm14"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-tiles", default="",
                    help="batch workload: workers_per_cu,counts_tiles,fold_cols,rho_blocks,interleave[,staged] "
                         "instead of running the autotuner")
    ap.add_argument("--no-rho", action="store_true",
                    help="batch workload: coefficients only (LRE_NO_RHO), to attribute step (ii)'s share")
    ap.add_argument("--no-n12", action="store_true",
                    help="n14 workload: skip the n = 12 sub-record")
    ap.add_argument("--project-n", type=int, default=12, choices=range(1, 15), metavar="N",
                    help="qubits of the step-(iii) workload (--workload project)")
    ap.add_argument("--no-compare", action="store_true",
                    help="time only the headline Walsh path (no MFMA-vs-plain ratio)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one plain 1 GiB copy kernel (negation of a "
                         "float32 tensor) as the reference for rocprofv3 byte counters")
    ap.add_argument("--wht", default="plain", choices=["mfma", "plain"],
                    help="counts-pass Walsh transform for the headline run; the other one is "
                         "timed too for the MFMA-vs-plain ratio")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        raise SystemExit(2)

    import torch
    from paper_1602_08604_amd import lre

    torch.cuda.set_device(0)
    if args.workload == "project":
        return bench_project(args, torch, lre)
    if args.workload == "batch":
        return bench_batch(args, torch, lre)
    if args.workload == "stream15":
        return bench_stream(args, torch, lre)
    if args.workload == "povm14":
        return bench_povm(args, torch, lre)
    out = bench_estimate(args.workload, args, torch, lre, extras=True)
    if args.workload == "n14" and not args.no_n12:
        # the metric names n = 12 too: its step time beside the headline, from the same run
        torch.cuda.empty_cache()
        sub = bench_estimate("n12", args, torch, lre, extras=False)
        out["n12"] = {k: sub[k] for k in ("value", "unit", "ms_per_step", "step_ms", "whole_step_hbm_frac",
                                          "mfma_vs_plain", "config")}
        out["n12"]["counts_pass_roofline_frac"] = sub["roofline"]["frac"]
        out["n12"]["counts_pass_traffic"] = sub["roofline"]["traffic"]
    print(json.dumps(out), flush=True)


def bench_estimate(workload, args, torch, lre, extras):
    """One workload through lre_estimate: K timed steps of the headline counts-pass form
    and of the other form (MFMA vs plain), outputs of the two compared."""
    t_gen = time.time()
    n, counts, shots, nb, desc = make_workload(workload, torch)
    torch.cuda.synchronize()
    t_gen = time.time() - t_gen
    d = 1 << n
    coef = torch.empty(4 ** n, dtype=torch.float64, device="cuda:0")
    rho = torch.empty((d, d), dtype=torch.complex128, device="cuda:0")
    ws = torch.empty(lre.workspace_bytes(n, shots, 0), dtype=torch.uint8, device="cuda:0")
    print(f"[bench] workload {workload}: generated in {t_gen:.1f} s; workspace "
          f"{ws.numel() / 1e9:.2f} GB", file=sys.stderr, flush=True)

    def timed(flags):
        def step():
            lre.estimate(counts, shots, n_per_basis=nb, coef=coef, rho=rho, workspace=ws,
                         flags=flags, check=False)

        for _ in range(args.warmup):
            step()
        lre.check_flags("cuda:0")
        ev = StageEvents(args.steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            lre.set_stage_events(ev.ev[k])
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lre.set_stage_events(None)
        lre.check_flags("cuda:0")
        res = {"ms_step": (t1 - t0) * 1e3 / args.steps,
               "pass1": [ev.ms(k, 0, 1) for k in range(args.steps)],
               "step_i": [ev.ms(k, 0, 2) for k in range(args.steps)],
               "step_ii": [ev.ms(k, 2, 3) for k in range(args.steps)],
               "whole": [ev.ms(k, 0, 3) for k in range(args.steps)]}
        ev.close()
        mean = lambda v: sum(v) / len(v)
        print(f"[bench] {workload} flags={flags}: {args.steps} steps: {res['ms_step']:.3f} ms/step wall; counts pass "
              f"{mean(res['pass1']):.3f} ms, step (i) {mean(res['step_i']):.3f} ms, "
              f"step (ii) {mean(res['step_ii']):.3f} ms", file=sys.stderr, flush=True)
        return res

    mfma_ok = n >= 7
    head_flags = lre.LRE_WHT_MFMA if (args.wht == "mfma" and mfma_ok) else 0
    head = timed(head_flags)
    head_coef = coef.clone() if (mfma_ok and not args.no_compare) else None
    other = timed(0 if head_flags else lre.LRE_WHT_MFMA) if (mfma_ok and not args.no_compare) else None
    if args.copy_calibration and extras:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    ms_step = head["ms_step"]
    pass1, step_i, step_ii = head["pass1"], head["step_i"], head["step_ii"]
    graph = None
    if n <= 12:
        # the same step captured into a HIP graph and replayed (no launch gaps between
        # its kernels; the lines' value stays the eager rate)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            lre.estimate(counts, shots, n_per_basis=nb, coef=coef, rho=rho, workspace=ws, flags=head_flags,
                         check=False)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            lre.estimate(counts, shots, n_per_basis=nb, coef=coef, rho=rho, workspace=ws, flags=head_flags,
                         check=False)
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.replay()
        torch.cuda.synchronize()
        graph = {"ms_per_step": (time.perf_counter() - t0) * 1e3 / args.steps,
                 "how": "one lre_estimate captured into a HIP graph (torch.cuda.CUDAGraph), replayed per step"}
        lre.check_flags("cuda:0")
        print(f"[bench] {workload}: graph replay {graph['ms_per_step']:.4f} ms/step", file=sys.stderr, flush=True)
        del g

    cold = None
    if n <= 8:
        # cold caches: a 512 MB buffer touched before each timed call
        flush = torch.empty(1 << 27, dtype=torch.float32, device="cuda:0")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        cold_ms = []
        for _ in range(max(args.steps, 5)):
            flush.fill_(1.0)
            torch.cuda.synchronize()
            e0.record()
            lre.estimate(counts, shots, n_per_basis=nb, coef=coef, rho=rho, workspace=ws, flags=head_flags,
                         check=False)
            e1.record()
            torch.cuda.synchronize()
            cold_ms.append(e0.elapsed_time(e1))
        lre.check_flags("cuda:0")
        del flush
        cold = {"median_ms": statistics.median(cold_ms), "min_ms": min(cold_ms),
                "how": "512 MB buffer written before each call; events around the call"}

    n_counts = 3 ** n * d
    t_pass1 = sum(pass1) / len(pass1) / 1e3
    achieved = 2.0 * n_counts / t_pass1 / 1e9
    traffic = measured_traffic(workload)
    algo_bytes = 2.0 * n_counts + 8.0 * 4 ** n + 16.0 * 4 ** n
    out = {
        "metric": METRIC,
        "value": n_counts / (ms_step / 1e3),
        "unit": "counts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "shots": shots if shots else "per-basis",
                   "wht": "int8-mfma" if head_flags else "plain-int32", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fold_counts_stream_kernel (counts pass of step (i))",
                     "algorithmic_bytes_per_launch": 2.0 * n_counts},
        "end_to_end_s": ms_step / 1e3,
        "step_ms": {"counts_pass": t_pass1 * 1e3, "step_i": sum(step_i) / len(step_i),
                    "step_ii": sum(step_ii) / len(step_ii)},
        "whole_step_hbm_frac": algo_bytes / (ms_step / 1e3) / (HBM_PEAK_GBS * 1e9),
        "wht": "int8-mfma" if head_flags else "plain-int32",
        "mfma_vs_plain": None,
    }
    out["device_ms"] = {
        "whole_step": {"median": statistics.median(head["whole"]), "min": min(head["whole"])},
        "counts_pass": {"median": statistics.median(pass1), "min": min(pass1)},
        "how": "HIP events the library records at stage boundaries, per timed step"}
    if cold is not None:
        out["cold_cache"] = cold
    if graph is not None:
        out["graph_replay"] = graph
    if other is not None:
        mfma, plain = (head, other) if head_flags else (other, head)
        mean = lambda v: sum(v) / len(v)
        # int8 work of the MFMA form: H_64 on two byte limbs = 64 multiply-adds per limb per count
        mfma_tops = 2.0 * 64 * 2 * n_counts / (mean(mfma["pass1"]) / 1e3) / 1e12
        # the two forms' coefficients, compared here (exact integers with uniform shots;
        # binary64 sums in LDS-atomic order with per-basis totals)
        diff = (coef - head_coef).abs().max().item()
        same = bool(torch.equal(coef, head_coef))
        del head_coef
        out["mfma_vs_plain"] = {
            "mfma_int8_tops": mfma_tops, "mfma_int8_peak_tops": 5000.0, "mfma_frac": mfma_tops / 5000.0,
            "counts_pass_speedup": mean(plain["pass1"]) / mean(mfma["pass1"]),
            "step_speedup": plain["ms_step"] / mfma["ms_step"],
            "plain_counts_pass_ms": mean(plain["pass1"]), "mfma_counts_pass_ms": mean(mfma["pass1"]),
            "plain_ms_per_step": plain["ms_step"], "mfma_ms_per_step": mfma["ms_step"],
            "coef_bit_identical": same, "coef_max_abs_diff": diff}
    if extras and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(workload, n, shots, counts, coef)
    if extras and not args.no_compare:
        del counts, ws, rho, coef, nb
        torch.cuda.empty_cache()
        out["hbm_measured"] = measured_hbm(torch, lre)
        out["compute_measured"] = measured_compute(torch, lre)
        # the counts pass against the device's measured streaming-read rate as well
        out["roofline"]["frac_of_measured_read"] = achieved / out["hbm_measured"]["stream_read_gbs"]
    return out


if __name__ == "__main__":
    main()
