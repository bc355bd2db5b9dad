"""Python binding of the gfx950 LRE library (include/lre.h) via ctypes.

Argument marshalling only: tensors are checked for dtype, device, shape and
contiguity, and their device pointers are handed to the C ABI together with the
current HIP stream.  Every step of the computation runs in the HIP kernels of
liblre.so; there is no fallback, and a missing library raises LreError.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "liblre.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "lre.h")

LRE_OK = 0
LRE_E_ARG = 1
LRE_E_WORKSPACE = 2
LRE_E_HIP = 3
LRE_E_SHOTS = 4
LRE_E_EMPTY_BASIS = 5
LRE_E_UNSUPPORTED = 6
LRE_E_TIMEOUT = 7
LRE_E_EIG = 8

LRE_NO_RHO = 0x1
LRE_RHO_FP32 = 0x2
LRE_WHT_MFMA = 0x4
LRE_STREAM_HOST = 0x8
LRE_STREAM_MAX_QUBITS = 15
LRE_MAX_QUBITS = 14
LRE_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024
LRE_BATCH_MAX_QUBITS = 9


class lre_instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("counts", ctypes.c_void_p), ("shots", ctypes.c_uint64),
                ("n_per_basis", ctypes.c_void_p), ("coef", ctypes.c_void_p), ("rho", ctypes.c_void_p)]


class lre_batch_tiles(ctypes.Structure):
    _fields_ = [("workers_per_cu", ctypes.c_int), ("counts_tiles", ctypes.c_int),
                ("fold_cols", ctypes.c_int), ("rho_blocks", ctypes.c_int), ("interleave", ctypes.c_int),
                ("staged", ctypes.c_int)]


class LreError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = status_str(status) if _lib_handle is not None else f"status {status}"
        super().__init__(f"{what}: {msg}" if what else msg)


_lib_handle = None


def lib():
    """The loaded liblre.so (raises LreError if it has not been built)."""
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(LIB_PATH):
            raise LreError(LRE_E_UNSUPPORTED, f"HIP library not built: {LIB_PATH} "
                                              "(run python -m paper_1602_08604_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, I, U32, U64, SZ, I64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                   ctypes.c_size_t, ctypes.c_int64)
        L.lre_create.argtypes = [ctypes.POINTER(P), I]
        L.lre_create.restype = I
        L.lre_destroy.argtypes = [P]
        L.lre_destroy.restype = None
        L.lre_status_str.argtypes = [I]
        L.lre_status_str.restype = ctypes.c_char_p
        L.lre_workspace_bytes.argtypes = [I, U64, U32]
        L.lre_workspace_bytes.restype = SZ
        L.lre_estimate.argtypes = [P, I, P, U64, P, P, P, P, SZ, U32, P]
        L.lre_estimate.restype = I
        L.lre_estimate_noalloc.argtypes = [P, I, P, U64, P, P, P, U32, P]
        L.lre_estimate_noalloc.restype = I
        L.lre_check.argtypes = [P, P]
        L.lre_check.restype = I
        L.lre_pauli_sums.argtypes = [P, I, P, U64, P, P, SZ, U32, P]
        L.lre_pauli_sums.restype = I
        L.lre_signed_sums.argtypes = [P, I, P, P, I64, P, U32, P]
        L.lre_signed_sums.restype = I
        L.lre_set_stage_events.argtypes = [P, ctypes.POINTER(P), I]
        L.lre_set_stage_events.restype = I
        L.lre_batch_plan.argtypes = [P, ctypes.POINTER(lre_instance), I, U32, ctypes.POINTER(P)]
        L.lre_batch_plan.restype = I
        L.lre_batch_workspace_bytes.argtypes = [P]
        L.lre_batch_workspace_bytes.restype = SZ
        L.lre_batch_set_tiles.argtypes = [P, ctypes.POINTER(lre_batch_tiles)]
        L.lre_batch_set_tiles.restype = I
        L.lre_batch_get_tiles.argtypes = [P, ctypes.POINTER(lre_batch_tiles), ctypes.POINTER(I)]
        L.lre_batch_get_tiles.restype = I
        L.lre_batch_tune.argtypes = [P, P, SZ, I, ctypes.POINTER(ctypes.c_double), P]
        L.lre_batch_tune.restype = I
        L.lre_batch_run.argtypes = [P, P, SZ, P]
        L.lre_batch_run.restype = I
        L.lre_project_workspace_bytes.argtypes = [I]
        L.lre_project_workspace_bytes.restype = SZ
        L.lre_project.argtypes = [P, I, P, P, P, P, SZ, P]
        L.lre_project.restype = I
        L.lre_stream_read.argtypes = [P, SZ, P, P]
        L.lre_stream_read.restype = I
        L.lre_stream_copy.argtypes = [P, P, SZ, P]
        L.lre_stream_copy.restype = I
        for name in ("lre_peak_valu_i32", "lre_peak_mfma_i8"):
            getattr(L, name).argtypes = [I, P, ctypes.POINTER(ctypes.c_double), P]
            getattr(L, name).restype = I
        L.lre_batch_destroy.argtypes = [P]
        L.lre_batch_destroy.restype = None
        L.lre_stream_create.argtypes = [P, I, I, U64, U32, ctypes.POINTER(P)]
        L.lre_stream_create.restype = I
        L.lre_stream_workspace_bytes.argtypes = [P]
        L.lre_stream_workspace_bytes.restype = SZ
        L.lre_stream_begin.argtypes = [P, P, P, SZ, P]
        L.lre_stream_begin.restype = I
        L.lre_stream_push.argtypes = [P, I64, P, P, P, SZ, P]
        L.lre_stream_push.restype = I
        L.lre_stream_push_host.argtypes = [P, I64, P, P, P, SZ, P]
        L.lre_stream_push_host.restype = I
        L.lre_stream_finish.argtypes = [P, P, P, SZ, P]
        L.lre_stream_finish.restype = I
        L.lre_stream_destroy.argtypes = [P]
        L.lre_stream_destroy.restype = None
        L.lre_povm_workspace_bytes.argtypes = [I, U32]
        L.lre_povm_workspace_bytes.restype = SZ
        L.lre_povm_estimate.argtypes = [P, I, P, P, P, P, P, SZ, U32, P]
        L.lre_povm_estimate.restype = I
        _lib_handle = L
    return _lib_handle


def declared_symbols(header: str = HEADER_PATH):
    """Function names declared in include/lre.h."""
    with open(header) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(lre_\w+)\s*\(", text, re.M)))


def status_str(status: int) -> str:
    return lib().lre_status_str(int(status)).decode()


def _ok(status: int, what: str):
    if status != LRE_OK:
        raise LreError(status, what)


_contexts: dict[int, int] = {}


def context(device: int | None = None) -> int:
    """lre_ctx* for a device (created once per process)."""
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _contexts:
        h = ctypes.c_void_p()
        _ok(lib().lre_create(ctypes.byref(h), dev), "lre_create")
        _contexts[dev] = h.value
    return _contexts[dev]


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _num_qubits(counts: torch.Tensor) -> int:
    if counts.dim() != 2:
        raise ValueError("counts must be 2-D (3^n, 2^n)")
    d = counts.shape[1]
    n = d.bit_length() - 1
    if d != 1 << n or counts.shape[0] != 3 ** n or not 1 <= n <= LRE_MAX_QUBITS:
        raise ValueError(f"counts shape {tuple(counts.shape)} is not (3^n, 2^n) with 1 <= n <= 14")
    return n


def _check_counts(counts: torch.Tensor) -> int:
    if counts.dtype not in (torch.uint16, torch.int16):
        raise TypeError("counts must be uint16 (int16 is reinterpreted bitwise)")
    if not counts.is_cuda or not counts.is_contiguous():
        raise ValueError("counts must be a contiguous device tensor")
    return _num_qubits(counts)


def workspace_bytes(n: int, shots: int, flags: int = 0) -> int:
    return int(lib().lre_workspace_bytes(int(n), int(shots), int(flags)))


def estimate(counts: torch.Tensor, shots: int, n_per_basis: torch.Tensor | None = None,
             flags: int = 0, coef: torch.Tensor | None = None, rho: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None, check: bool = True):
    """lre_estimate: (coef float64 [4^n], rho complex [2^n, 2^n] or None)."""
    n = _check_counts(counts)
    dev = counts.device
    d = 1 << n
    if coef is None:
        coef = torch.empty(4 ** n, dtype=torch.float64, device=dev)
    want_rho = not (flags & LRE_NO_RHO)
    if want_rho and rho is None:
        rho = torch.empty((d, d), dtype=torch.complex64 if flags & LRE_RHO_FP32 else torch.complex128,
                          device=dev)
    if n_per_basis is not None:
        if n_per_basis.dtype not in (torch.int32, torch.uint32) or not n_per_basis.is_cuda \
                or n_per_basis.numel() != 3 ** n or not n_per_basis.is_contiguous():
            raise ValueError("n_per_basis must be a contiguous 32-bit device tensor of length 3^n")
    wsb = workspace_bytes(n, shots, flags)
    if workspace is None:
        workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    st = lib().lre_estimate(
        ctypes.c_void_p(context(dev.index)), n, ctypes.c_void_p(counts.data_ptr()), int(shots),
        ctypes.c_void_p(n_per_basis.data_ptr() if n_per_basis is not None else None),
        ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(rho.data_ptr() if want_rho else None),
        ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), int(flags),
        ctypes.c_void_p(_stream(dev)))
    _ok(st, "lre_estimate")
    if check:
        check_flags(dev)
    return coef, rho


def estimate_noalloc(counts: torch.Tensor, shots: int, coef: torch.Tensor, rho: torch.Tensor | None,
                     n_per_basis: torch.Tensor | None = None, flags: int = 0, check: bool = True):
    """lre_estimate_noalloc: lre_estimate into caller-given outputs with the library's
    static device scratch as workspace (no device allocation by the call)."""
    n = _check_counts(counts)
    dev = counts.device
    want_rho = not (flags & LRE_NO_RHO)
    if coef.dtype != torch.float64 or coef.numel() != 4 ** n or not coef.is_contiguous():
        raise ValueError("coef must be a contiguous float64 tensor of length 4^n")
    if want_rho and (rho is None or rho.numel() != 4 ** n or not rho.is_contiguous()):
        raise ValueError("rho must be a contiguous 2^n x 2^n complex tensor")
    if n_per_basis is not None and (n_per_basis.dtype not in (torch.int32, torch.uint32)
                                    or n_per_basis.numel() != 3 ** n or not n_per_basis.is_contiguous()):
        raise ValueError("n_per_basis must be a contiguous 32-bit device tensor of length 3^n")
    st = lib().lre_estimate_noalloc(
        ctypes.c_void_p(context(dev.index)), n, ctypes.c_void_p(counts.data_ptr()), int(shots),
        ctypes.c_void_p(n_per_basis.data_ptr() if n_per_basis is not None else None),
        ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(rho.data_ptr() if want_rho else None),
        int(flags), ctypes.c_void_p(_stream(dev)))
    _ok(st, "lre_estimate_noalloc")
    if check:
        check_flags(dev)
    return coef, rho


def povm_estimate(counts: torch.Tensor, G, flags: int = 0, coef: torch.Tensor | None = None,
                  rho: torch.Tensor | None = None, workspace: torch.Tensor | None = None, check: bool = True):
    """lre_povm_estimate (reduced measurement set): counts uint16 device [4^n] (or any
    contiguous shape with 4^n elements), G the 4 x 4 Pauli components Tr(E_j sigma_a) of
    the per-qubit operators (array-like or float64 device tensor).  Returns (coef, rho)."""
    if counts.dtype not in (torch.uint16, torch.int16) or not counts.is_cuda or not counts.is_contiguous():
        raise ValueError("counts must be a contiguous uint16 device tensor")
    m = counts.numel()
    n = (m.bit_length() - 1) // 2
    if m != 4 ** n or not 1 <= n <= LRE_MAX_QUBITS:
        raise ValueError("counts must hold 4^n outcomes, 1 <= n <= 14")
    dev = counts.device
    g = torch.as_tensor(G, dtype=torch.float64).to(dev).contiguous()
    if g.numel() != 16:
        raise ValueError("G must be 4 x 4")
    d = 1 << n
    if coef is None:
        coef = torch.empty(4 ** n, dtype=torch.float64, device=dev)
    want_rho = not (flags & LRE_NO_RHO)
    if want_rho and rho is None:
        rho = torch.empty((d, d), dtype=torch.complex64 if flags & LRE_RHO_FP32 else torch.complex128,
                          device=dev)
    wsb = int(lib().lre_povm_workspace_bytes(n, int(flags)))
    if workspace is None:
        workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    _ok(lib().lre_povm_estimate(ctypes.c_void_p(context(dev.index)), n, ctypes.c_void_p(counts.data_ptr()),
                                ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(coef.data_ptr()),
                                ctypes.c_void_p(rho.data_ptr() if want_rho else None),
                                ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), int(flags),
                                ctypes.c_void_p(_stream(dev))), "lre_povm_estimate")
    if check:
        check_flags(dev)
    return coef, rho


def project(mu: torch.Tensor, rho: torch.Tensor | None = None, eigvals: torch.Tensor | None = None,
            workspace: torch.Tensor | None = None, check: bool = True):
    """lre_project (step (iii)): (rho complex128 [d, d] closest physical state, eigenvalues
    of mu ascending float64 [d])."""
    if mu.dtype != torch.complex128 or not mu.is_cuda or not mu.is_contiguous() or mu.dim() != 2 \
            or mu.shape[0] != mu.shape[1]:
        raise ValueError("mu must be a contiguous complex128 square device tensor")
    d = mu.shape[0]
    n = d.bit_length() - 1
    if d != 1 << n:
        raise ValueError("mu must be 2^n x 2^n")
    dev = mu.device
    if rho is None:
        rho = torch.empty_like(mu)
    if eigvals is None:
        eigvals = torch.empty(d, dtype=torch.float64, device=dev)
    wsb = lib().lre_project_workspace_bytes(n)
    if workspace is None:
        workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    st = lib().lre_project(ctypes.c_void_p(context(dev.index)), n, ctypes.c_void_p(mu.data_ptr()),
                           ctypes.c_void_p(rho.data_ptr()), ctypes.c_void_p(eigvals.data_ptr()),
                           ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), ctypes.c_void_p(_stream(dev)))
    _ok(st, "lre_project")
    if check:
        check_flags(dev)
    return rho, eigvals


def check_flags(device=None):
    """lre_check: synchronise the current stream and raise on a data error flag."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    _ok(lib().lre_check(ctypes.c_void_p(context(dev.index)), ctypes.c_void_p(_stream(dev))), "lre_check")


def pauli_sums(counts: torch.Tensor, shots: int, flags: int = 0, T: torch.Tensor | None = None,
               workspace: torch.Tensor | None = None, check: bool = True) -> torch.Tensor:
    """lre_pauli_sums: exact int64 numerators T_i of eq. (3) (uniform shots)."""
    n = _check_counts(counts)
    dev = counts.device
    if T is None:
        T = torch.empty(4 ** n, dtype=torch.int64, device=dev)
    wsb = workspace_bytes(n, shots, flags | LRE_NO_RHO)
    if workspace is None:
        workspace = torch.empty(max(wsb, 1), dtype=torch.uint8, device=dev)
    st = lib().lre_pauli_sums(ctypes.c_void_p(context(dev.index)), n, ctypes.c_void_p(counts.data_ptr()),
                              int(shots), ctypes.c_void_p(T.data_ptr()),
                              ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), int(flags),
                              ctypes.c_void_p(_stream(dev)))
    _ok(st, "lre_pauli_sums")
    if check:
        check_flags(dev)
    return T


def signed_sums(counts: torch.Tensor, bases: torch.Tensor, flags: int = 0,
                check: bool = True) -> torch.Tensor:
    """lre_signed_sums: int32 [len(bases), 2^n] Walsh sums of the selected rows."""
    n = _check_counts(counts)
    dev = counts.device
    if bases.dtype != torch.int64 or not bases.is_cuda or not bases.is_contiguous():
        raise ValueError("bases must be a contiguous int64 device tensor")
    out = torch.empty((bases.numel(), 1 << n), dtype=torch.int32, device=dev)
    st = lib().lre_signed_sums(ctypes.c_void_p(context(dev.index)), n, ctypes.c_void_p(counts.data_ptr()),
                               ctypes.c_void_p(bases.data_ptr()), bases.numel(),
                               ctypes.c_void_p(out.data_ptr()), int(flags), ctypes.c_void_p(_stream(dev)))
    _ok(st, "lre_signed_sums")
    if check:
        check_flags(dev)
    return out


def stream_read(buf: torch.Tensor, sink: torch.Tensor) -> None:
    """lre_stream_read over the bytes of a contiguous device tensor (diagnostic)."""
    if not (buf.is_cuda and buf.is_contiguous() and sink.is_cuda and sink.dtype == torch.int32):
        raise ValueError("buf: contiguous device tensor; sink: int32 device tensor")
    _ok(lib().lre_stream_read(ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                              ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(_stream(buf.device))),
        "lre_stream_read")


def stream_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    """lre_stream_copy between two contiguous device tensors of equal size (diagnostic)."""
    nbytes = src.numel() * src.element_size()
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()
            and dst.numel() * dst.element_size() == nbytes):
        raise ValueError("src, dst: contiguous device tensors of equal size")
    _ok(lib().lre_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nbytes,
                              ctypes.c_void_p(_stream(src.device))), "lre_stream_copy")


def peak_rate(kind: str, iters: int, sink: torch.Tensor) -> float:
    """lre_peak_valu_i32 (kind "valu_i32") or lre_peak_mfma_i8 (kind "mfma_i8"): enqueue
    one launch on sink's device and return the number of operations it performs."""
    if not (sink.is_cuda and sink.dtype == torch.int32):
        raise ValueError("sink: int32 device tensor")
    fn = {"valu_i32": lib().lre_peak_valu_i32, "mfma_i8": lib().lre_peak_mfma_i8}[kind]
    ops = ctypes.c_double(0.0)
    _ok(fn(int(iters), ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ops), ctypes.c_void_p(_stream(sink.device))),
        f"lre_peak_{kind}")
    return ops.value


def set_stage_events(events, device=None):
    """lre_set_stage_events: raw hipEvent_t handles (ints) or None to disable."""
    ctx = ctypes.c_void_p(context(device))
    if not events:
        _ok(lib().lre_set_stage_events(ctx, None, 0), "lre_set_stage_events")
        return
    arr = (ctypes.c_void_p * len(events))(*events)
    _ok(lib().lre_set_stage_events(ctx, arr, len(events)), "lre_set_stage_events")


class Batch:
    """lre_batch_*: many instances (n <= 9) in one persistent launch.

    counts: list of uint16 device tensors [3^n, 2^n]; shots: list of ints (0 = per-basis
    totals, then n_per_basis[j] is a 32-bit device tensor [3^n] or None for the row
    sums).  Output tensors are allocated unless given (coef float64 [4^n]; rho complex
    [2^n, 2^n] unless LRE_NO_RHO).  The plan keeps references to every tensor it points
    to."""

    def __init__(self, counts, shots, flags=0, coefs=None, rhos=None, n_per_basis=None):
        if len(counts) != len(shots) or not counts:
            raise ValueError("counts and shots must be non-empty lists of equal length")
        self.flags = int(flags)
        self.counts = list(counts)
        self.shots = [int(x) for x in shots]
        self.nb = list(n_per_basis) if n_per_basis is not None else [None] * len(self.counts)
        if len(self.nb) != len(self.counts):
            raise ValueError("n_per_basis must have one entry per instance")
        dev = self.counts[0].device
        self.device = dev
        want_rho = not (flags & LRE_NO_RHO)
        cdt = torch.complex64 if flags & LRE_RHO_FP32 else torch.complex128
        self.n = [_check_counts(c) for c in self.counts]
        self.coefs = list(coefs) if coefs is not None else [
            torch.empty(4 ** n, dtype=torch.float64, device=dev) for n in self.n]
        if want_rho:
            self.rhos = list(rhos) if rhos is not None else [
                torch.empty((1 << n, 1 << n), dtype=cdt, device=dev) for n in self.n]
        else:
            self.rhos = [None] * len(self.n)
        arr = (lre_instance * len(self.n))()
        for j, n in enumerate(self.n):
            arr[j].n = n
            arr[j].counts = self.counts[j].data_ptr()
            arr[j].shots = self.shots[j]
            nb = self.nb[j]
            if nb is not None and (nb.dtype not in (torch.int32, torch.uint32) or not nb.is_cuda
                                   or nb.numel() != 3 ** n or not nb.is_contiguous()):
                raise ValueError("n_per_basis entries must be contiguous 32-bit device tensors of length 3^n")
            arr[j].n_per_basis = nb.data_ptr() if nb is not None else None
            arr[j].coef = self.coefs[j].data_ptr()
            arr[j].rho = self.rhos[j].data_ptr() if self.rhos[j] is not None else None
        h = ctypes.c_void_p()
        _ok(lib().lre_batch_plan(ctypes.c_void_p(context(dev.index)), arr, len(self.n), self.flags,
                                 ctypes.byref(h)), "lre_batch_plan")
        self._h = h.value
        self._ws = None

    @property
    def workspace_bytes(self) -> int:
        return int(lib().lre_batch_workspace_bytes(ctypes.c_void_p(self._h)))

    def workspace(self):
        if self._ws is None or self._ws.numel() < self.workspace_bytes:
            self._ws = torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device=self.device)
        return self._ws

    def run(self, check: bool = False):
        ws = self.workspace()
        _ok(lib().lre_batch_run(ctypes.c_void_p(self._h), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                ctypes.c_void_p(_stream(self.device))), "lre_batch_run")
        if check:
            check_flags(self.device)
        return self.coefs, self.rhos

    def tune(self, reps: int = 3) -> float:
        ws = self.workspace()
        best = ctypes.c_double()
        _ok(lib().lre_batch_tune(ctypes.c_void_p(self._h), ctypes.c_void_p(ws.data_ptr()), ws.numel(), int(reps),
                                 ctypes.byref(best), ctypes.c_void_p(_stream(self.device))), "lre_batch_tune")
        return best.value

    @property
    def tiles(self) -> dict:
        t = lre_batch_tiles()
        k = ctypes.c_int()
        _ok(lib().lre_batch_get_tiles(ctypes.c_void_p(self._h), ctypes.byref(t), ctypes.byref(k)),
            "lre_batch_get_tiles")
        return {"workers_per_cu": t.workers_per_cu, "counts_tiles": t.counts_tiles, "fold_cols": t.fold_cols,
                "rho_blocks": t.rho_blocks, "interleave": t.interleave, "staged": t.staged, "items": k.value}

    def set_tiles(self, workers_per_cu, counts_tiles, fold_cols, rho_blocks, interleave, staged=0):
        t = lre_batch_tiles(workers_per_cu, counts_tiles, fold_cols, rho_blocks, interleave, staged)
        _ok(lib().lre_batch_set_tiles(ctypes.c_void_p(self._h), ctypes.byref(t)), "lre_batch_set_tiles")

    def close(self):
        if getattr(self, "_h", None):
            lib().lre_batch_destroy(ctypes.c_void_p(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    """lre_stream_*: an estimate whose counts arrive slab by slab (slab k: the 3^(n-h)
    bases whose top h qubits carry the letters of k's base-3 digits, uint16 [3^(n-h), 2^n]).

    begin() clears the coefficient accumulator; push(k, counts) takes a device slab,
    push_host(k, counts) a host (CPU) tensor, copied by the library into its staging
    slab (flags must include LRE_STREAM_HOST); finish() returns (coef, rho)."""

    def __init__(self, n: int, h: int, shots: int, flags: int = 0, device=None):
        self.n, self.h, self.shots, self.flags = int(n), int(h), int(shots), int(flags)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device) \
            if not isinstance(device, torch.device) else device
        self.rows = 3 ** (self.n - self.h)
        hdl = ctypes.c_void_p()
        _ok(lib().lre_stream_create(ctypes.c_void_p(context(self.device.index)), self.n, self.h, self.shots,
                                    self.flags, ctypes.byref(hdl)), "lre_stream_create")
        self._h = hdl.value
        self._ws = None
        self.coef = None

    @property
    def workspace_bytes(self) -> int:
        return int(lib().lre_stream_workspace_bytes(ctypes.c_void_p(self._h)))

    def workspace(self):
        if self._ws is None or self._ws.numel() < self.workspace_bytes:
            self._ws = torch.empty(max(1, self.workspace_bytes), dtype=torch.uint8, device=self.device)
        return self._ws

    def _args(self):
        ws = self.workspace()
        return ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(_stream(self.device))

    def begin(self, coef: torch.Tensor | None = None) -> torch.Tensor:
        if coef is None:
            coef = torch.empty(4 ** self.n, dtype=torch.float64, device=self.device)
        if coef.dtype != torch.float64 or coef.numel() != 4 ** self.n or not coef.is_contiguous():
            raise ValueError("coef must be a contiguous float64 device tensor of length 4^n")
        self.coef = coef
        _ok(lib().lre_stream_begin(ctypes.c_void_p(self._h), ctypes.c_void_p(coef.data_ptr()), *self._args()),
            "lre_stream_begin")
        return coef

    def _check_slab(self, counts, nb, host):
        if counts.dtype not in (torch.uint16, torch.int16) or tuple(counts.shape) != (self.rows, 1 << self.n) \
                or not counts.is_contiguous() or counts.is_cuda == host:
            raise ValueError(f"slab must be a contiguous uint16 {'host' if host else 'device'} tensor "
                             f"of shape ({self.rows}, {1 << self.n})")
        if nb is not None and (nb.dtype not in (torch.int32, torch.uint32) or nb.numel() != self.rows
                               or not nb.is_contiguous() or nb.is_cuda == host):
            raise ValueError("n_per_basis must be a contiguous 32-bit tensor of length 3^(n-h) beside the slab")

    def push(self, slab: int, counts: torch.Tensor, n_per_basis: torch.Tensor | None = None):
        self._check_slab(counts, n_per_basis, host=False)
        _ok(lib().lre_stream_push(ctypes.c_void_p(self._h), int(slab), ctypes.c_void_p(counts.data_ptr()),
                                  ctypes.c_void_p(n_per_basis.data_ptr() if n_per_basis is not None else None),
                                  *self._args()), "lre_stream_push")

    def push_host(self, slab: int, counts: torch.Tensor, n_per_basis: torch.Tensor | None = None):
        self._check_slab(counts, n_per_basis, host=True)
        _ok(lib().lre_stream_push_host(ctypes.c_void_p(self._h), int(slab), ctypes.c_void_p(counts.data_ptr()),
                                       ctypes.c_void_p(n_per_basis.data_ptr() if n_per_basis is not None else None),
                                       *self._args()), "lre_stream_push_host")

    def finish(self, rho: torch.Tensor | None = None, check: bool = True):
        want_rho = not (self.flags & LRE_NO_RHO)
        d = 1 << self.n
        if want_rho and rho is None:
            rho = torch.empty((d, d), dtype=torch.complex64 if self.flags & LRE_RHO_FP32 else torch.complex128,
                              device=self.device)
        _ok(lib().lre_stream_finish(ctypes.c_void_p(self._h), ctypes.c_void_p(rho.data_ptr() if want_rho else None),
                                    *self._args()), "lre_stream_finish")
        if check:
            check_flags(self.device)
        coef, self.coef = self.coef, None
        return coef, rho

    def close(self):
        if getattr(self, "_h", None):
            lib().lre_stream_destroy(ctypes.c_void_p(self._h))
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
