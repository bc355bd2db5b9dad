"""Device-side input generation (torch tensors on the GPU)."""
from __future__ import annotations

import ctypes
import os

import torch

from .build import LIB

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"input generator not built: {LIB} (python -m tomo_inputs.build)")
        L = ctypes.CDLL(LIB)
        L.tomo_gen_philox_counts.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_int64,
                                             ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p]
        L.tomo_gen_philox_counts.restype = ctypes.c_int
        L.tomo_gen_philox_counts_paired.argtypes = L.tomo_gen_philox_counts.argtypes
        L.tomo_gen_philox_counts_paired.restype = ctypes.c_int
        _lib = L
    return _lib


def philox_counts(n: int, seed: int, b_begin: int = 0, b_count: int | None = None,
                  counts: torch.Tensor | None = None, nb: torch.Tensor | None = None,
                  device="cuda", paired: bool = False):
    """Rows [b_begin, b_begin + b_count) of the Philox workload: (counts uint16 [rows, 2^n],
    nb int32 [rows]), generated on the device.  paired: outcome 2k + 1 becomes 12 minus
    outcome 2k, so every basis totals 12 * 2^(n-1) (a uniform-shot workload)."""
    b_count = 3 ** n - b_begin if b_count is None else b_count
    if counts is None:
        counts = torch.empty((b_count, 1 << n), dtype=torch.uint16, device=device)
    if nb is None:
        nb = torch.empty(b_count, dtype=torch.int32, device=device)
    st = torch.cuda.current_stream(counts.device).cuda_stream
    gen = _load().tomo_gen_philox_counts_paired if paired else _load().tomo_gen_philox_counts
    rc = gen(n, seed, b_begin, b_count, ctypes.c_void_p(counts.data_ptr()), ctypes.c_void_p(nb.data_ptr()),
             ctypes.c_void_p(st))
    if rc != 0:
        raise RuntimeError(f"tomo_gen_philox_counts failed ({rc})")
    return counts, nb


def ghz_multinomial_counts(n: int, p_dep: float, shots: int, seed: int, device="cuda",
                           slab: int = 8192) -> torch.Tensor:
    """Multinomial counts (shots per basis) of rho = (1-p)|GHZ><GHZ| + p I/2^n, sampled on the
    device with torch.multinomial and a seeded torch.Generator, slab by slab of bases.
    Returns uint16 [3^n, 2^n].  The same (n, p_dep, shots, seed, slab) on the same device
    type reproduces the same counts."""
    from . import BASIS_BRAS
    B, d = 3 ** n, 2 ** n
    if shots > 65535:
        raise ValueError("shots must fit uint16 counts")
    out = torch.empty((B, d), dtype=torch.uint16, device=device)
    bras = torch.from_numpy(BASIS_BRAS).to(device)                      # (3, 2, 2)
    s = torch.arange(d, device=device)
    bits = torch.stack([(s >> (n - 1 - k)) & 1 for k in range(n)], dim=1)  # (d, n)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    for b0 in range(0, B, slab):
        b1 = min(B, b0 + slab)
        b = torch.arange(b0, b1, device=device)
        a0 = torch.ones((b1 - b0, d), dtype=torch.complex128, device=device)
        a1 = torch.ones_like(a0)
        for k in range(n):
            u = bras[(b // 3 ** (n - 1 - k)) % 3]                           # (nb, 2, 2)
            uk = u[:, bits[:, k], :]                                         # (nb, d, 2)
            a0 *= uk[:, :, 0]
            a1 *= uk[:, :, 1]
        p = (1.0 - p_dep) * 0.5 * (a0 + a1).abs() ** 2 + p_dep / d
        idx = torch.multinomial(p, shots, replacement=True, generator=g)   # (nb, shots)
        cnt = torch.zeros((b1 - b0, d), dtype=torch.int32, device=device)
        cnt.scatter_add_(1, idx, torch.ones_like(idx, dtype=torch.int32))
        out[b0:b1] = cnt.to(torch.uint16)
        del a0, a1, p, idx, cnt
    return out


def rotated_amplitudes(n: int, psi: torch.Tensor) -> torch.Tensor:
    """(U_b psi)_s for every basis b: complex128 [3^n, 2^n] on psi's device (the same
    axis-by-axis contraction as tomo_inputs.rotated_amplitudes)."""
    from . import BASIS_BRAS
    U = torch.from_numpy(BASIS_BRAS).to(psi.device)                    # (3, 2, 2)
    t = psi.reshape((1,) + (2,) * n).contiguous()
    for k in range(n):
        t = torch.tensordot(U, t, dims=([2], [1 + k]))                 # (3, 2, 3^k, rest)
        t = torch.movedim(t, 2, 0)                                     # (3^k, 3, 2, rest)
        t = torch.movedim(t, 2, 2 + k)
        t = t.reshape((-1,) + tuple(t.shape[2:])).contiguous()
    return t.reshape(3 ** n, 2 ** n)


def multinomial_rows(p: torch.Tensor, shots: int, generator: torch.Generator, slab: int = 2048) -> torch.Tensor:
    """One multinomial draw of `shots` per row of p (rows need not be normalised), as
    uint16 counts, sampled with torch.multinomial slab by slab."""
    if shots > 65535:
        raise ValueError("shots must fit uint16 counts")
    B, d = p.shape
    out = torch.empty((B, d), dtype=torch.uint16, device=p.device)
    for b0 in range(0, B, slab):
        b1 = min(B, b0 + slab)
        idx = torch.multinomial(p[b0:b1], shots, replacement=True, generator=generator)
        cnt = torch.zeros((b1 - b0, d), dtype=torch.int32, device=p.device)
        cnt.scatter_add_(1, idx, torch.ones_like(idx, dtype=torch.int32))
        out[b0:b1] = cnt.to(torch.uint16)
        del idx, cnt
    return out


def haar_multinomial_counts(n: int, shots: int, seed: int, device="cuda") -> torch.Tensor:
    """Counts of a Haar-random pure state: the state from numpy default_rng(seed)
    (tomo_inputs.haar_state), Born probabilities of every basis on the device, then
    `shots` multinomial draws per basis from a torch.Generator seeded with `seed`.
    uint16 [3^n, 2^n]."""
    import numpy as np
    from . import haar_state
    psi = torch.from_numpy(haar_state(n, np.random.default_rng(seed))).to(device)
    p = rotated_amplitudes(n, psi).abs() ** 2
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return multinomial_rows(p, shots, g)
