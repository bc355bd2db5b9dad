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


def test_traffic_record_is_gated_by_source_hash_and_batch_shape(monkeypatch):
    """bench.py reports a committed HBM-traffic record only while the kernel sources hash
    to the recorded value and, for the batch, only for the work-item shape it was taken
    with."""
    import json
    import re
    from paper_1602_08604_amd import profsum
    with open(os.path.join(ROOT, "profiles", "traffic_batch_kernel_512_instances.json")) as f:
        rec = json.load(f)
    tiles = re.search(r"--batch-tiles (\S+) ", rec["command_fetch"]).group(1)
    monkeypatch.setattr(profsum, "kernel_source_hash", lambda workload="": rec["kernel_source_hash"])
    assert bench.measured_traffic("batch", tiles) == rec["hbm_bytes_per_launch"]
    other = ",".join(str(int(v) + (1 if k == 1 else 0)) for k, v in enumerate(tiles.split(",")))
    assert bench.measured_traffic("batch", other) is None
    monkeypatch.setattr(profsum, "kernel_source_hash", lambda workload="": "0" * 16)
    assert bench.measured_traffic("batch", tiles) is None
    assert bench.measured_traffic("n14") is None
