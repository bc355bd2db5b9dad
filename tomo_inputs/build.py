"""Build the on-device input generator (tomo_inputs/_lib/libtomo_gen.so) with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "philox_gen.hip")
LIB = os.path.join(HERE, "_lib", "libtomo_gen.so")
CSRC = os.path.join(HERE, "csrc", "philox_cpu.c")
CLIB = os.path.join(HERE, "_lib", "libtomo_cpu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build_cpu(force: bool = True) -> str:
    os.makedirs(os.path.dirname(CLIB), exist_ok=True)
    if force or not os.path.exists(CLIB) or os.path.getmtime(CLIB) < os.path.getmtime(CSRC):
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", CSRC,
                               "-o", CLIB + ".tmp"])
        os.replace(CLIB + ".tmp", CLIB)
    return CLIB


def build(force: bool = True, verbose: bool = False) -> str:
    build_cpu(force)
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    cmd = [HIPCC, *FLAGS, SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{err}")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
