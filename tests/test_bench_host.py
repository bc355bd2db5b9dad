"""Host-side parts of bench.py that need no GPU: the one-GPU refusal and the CPU
baseline leg (the oracle timed on a bounded sample)."""
import os
import subprocess
import sys

import numpy as np
import torch

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_leg_reports_the_oracle():
    n, shots = 4, 60
    rng = np.random.default_rng(3)
    # rows of a multinomial with `shots` draws each
    rows = np.stack([rng.multinomial(shots, np.full(2 ** n, 1.0 / 2 ** n)) for _ in range(3 ** n)])
    counts = torch.from_numpy(rows.astype(np.uint16))
    coef = torch.zeros(4 ** n, dtype=torch.float64)
    coef[0] = 1.0
    out = bench.cpu_baseline("n8", n, shots, counts, coef, budget_s=0.4)
    assert out["kind"] == "oracle" and out["unit"] == "counts/s"
    assert out["value"] > 0 and out["cores"] >= 1
    assert "random coefficients" in out["sample"]


def test_cpu_baseline_n14_all_cores_and_one():
    """The 14-qubit leg times the oracle on all host threads and on one."""
    out = bench.cpu_baseline("n14", 14, 0, None, None, budget_s=0.5)
    assert out["kind"] == "oracle" and out["value"] > 0 and out["cores"] >= 1
    one = out["one_core"]
    assert one["cores"] == 1 and one["value"] > 0
    assert "threads" in out["sample"] and "1 thread" in one["sample"]
