"""Host-side checks of the C ABI library (no GPU compute): it loads, exports every
symbol that include/lre.h declares, and its host-only entry points behave."""
import ctypes

import pytest

from paper_1602_08604_amd import lre as L


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    syms = L.declared_symbols()
    assert {"lre_create", "lre_destroy", "lre_estimate", "lre_check", "lre_pauli_sums",
            "lre_signed_sums", "lre_status_str", "lre_workspace_bytes"} <= set(syms)
    for s in syms:
        assert getattr(lib, s) is not None


def test_status_strings():
    for st in range(7):
        assert L.status_str(st) and L.status_str(st) != "unknown status"
    assert L.status_str(99) == "unknown status"


@pytest.mark.parametrize("n", [0, 15, -1])
def test_workspace_rejects_bad_n(n):
    assert L.workspace_bytes(n, 100) == 0


def test_workspace_sizes_are_sane():
    # counts pass output of the 14-qubit per-basis plan dominates: 6^7 * 4^7 binary64
    ws14 = L.workspace_bytes(14, 0)
    assert 6 ** 7 * 4 ** 7 * 8 <= ws14 < 60e9
    # small problems need little workspace
    assert L.workspace_bytes(3, 1000) < 1 << 20
    for n in range(1, 15):
        assert L.workspace_bytes(n, 1000) > 0 and L.workspace_bytes(n, 0) > 0


def test_create_rejects_null_out():
    assert L.lib().lre_create(None, 0) == L.LRE_E_ARG


def test_estimate_rejects_null_context():
    st = L.lib().lre_estimate(None, 4, ctypes.c_void_p(16), 10, None, ctypes.c_void_p(16),
                              None, None, 0, L.LRE_NO_RHO, None)
    assert st == L.LRE_E_ARG


def test_stream_diagnostics_reject_bad_arguments():
    lib = L.lib()
    buf = ctypes.c_void_p(4096)
    assert lib.lre_stream_read(None, 16, buf, None) == L.LRE_E_ARG
    assert lib.lre_stream_read(buf, 16, None, None) == L.LRE_E_ARG
    assert lib.lre_stream_read(ctypes.c_void_p(4100), 16, buf, None) == L.LRE_E_ARG   # misaligned
    assert lib.lre_stream_read(buf, 24, buf, None) == L.LRE_E_ARG                     # not 16-byte units
    assert lib.lre_stream_copy(buf, None, 16, None) == L.LRE_E_ARG
    assert lib.lre_stream_copy(buf, ctypes.c_void_p(8200), 16, None) == L.LRE_E_ARG
    assert lib.lre_stream_read(buf, 0, buf, None) == L.LRE_OK                         # nothing to do
