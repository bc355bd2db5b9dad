"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: integer sums bit-exact; coefficients with uniform shots bit-exact (both sides
divide the same exact integer once, IEEE round-to-nearest); per-basis coefficients
and rho within 1e-12 absolute; rho exactly Hermitian.
"""
import numpy as np
import pytest

import oracle
import tomo_inputs as ti
from tests import refs

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1602_08604_amd import lre as L  # noqa: E402

DEV = "cuda:0"
TOL = 1e-12


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _haar_counts(n, shots, seed):
    rng = np.random.default_rng(seed)
    return ti.multinomial_counts(ti.born_probs_pure(n, ti.haar_state(n, rng)), shots, rng)


def _walsh_coef_index(n, b, m):
    """Pauli index whose support is m for basis b: letter b_k + 1 where bit k of m is set."""
    i = 0
    for p in range(n):
        bp = (b // 3 ** p) % 3
        if (m >> p) & 1:
            i += (bp + 1) * 4 ** p
    return i


@pytest.mark.parametrize("n", list(range(1, 10)))
def test_pauli_sums_bit_exact(n):
    print(f"[pauli_sums n={n}]", flush=True)
    shots = 1000 if n < 9 else 200
    counts = _haar_counts(n, shots, 10 + n)
    T = L.pauli_sums(_dev(counts), shots).cpu().numpy()
    if n <= 8:
        np.testing.assert_array_equal(T, oracle.pauli_sums(n, counts))
    else:
        idx = np.random.default_rng(n).integers(0, 4 ** n, 3000)
        np.testing.assert_array_equal(T[idx], oracle.pauli_sums(n, counts, idx))


@pytest.mark.parametrize("n", list(range(1, 9)))
def test_estimate_uniform_bit_exact(n):
    print(f"[estimate uniform n={n}]", flush=True)
    shots = 777
    counts = _haar_counts(n, shots, 20 + n)
    coef, rho = L.estimate(_dev(counts), shots)
    coef, rho = coef.cpu().numpy(), rho.cpu().numpy()
    e_ref = oracle.coefs(n, counts, shots)
    np.testing.assert_array_equal(coef, e_ref)
    assert coef[0] == 1.0
    mu_ref = oracle.rho(n, e_ref)
    assert np.max(np.abs(rho - mu_ref)) <= TOL
    assert np.array_equal(rho, rho.conj().T)
    assert abs(np.trace(rho) - 1) <= TOL


@pytest.mark.parametrize("n,nb_given", [(2, True), (4, False), (6, True), (7, False), (8, True)])
def test_estimate_per_basis(n, nb_given):
    print(f"[estimate per-basis n={n} nb={nb_given}]", flush=True)
    rng = np.random.default_rng(30 + n)
    shots = rng.integers(100, 3000, size=3 ** n)
    counts = ti.multinomial_counts(ti.born_probs_pure(n, ti.haar_state(n, rng)), shots, rng)
    nb = _dev(counts.sum(axis=1).astype(np.int32)) if nb_given else None
    coef, rho = L.estimate(_dev(counts), 0, n_per_basis=nb)
    coef, rho = coef.cpu().numpy(), rho.cpu().numpy()
    e_ref = oracle.coefs(n, counts, 0)
    assert np.max(np.abs(coef - e_ref)) <= TOL
    # Frequencies c/N_b are formed with the rounded reciprocal of N_b, so the trace
    # coefficient is 1 only up to rounding (the oracle's is exactly 1).
    assert abs(coef[0] - 1.0) <= TOL
    assert np.max(np.abs(rho - oracle.rho(n, e_ref))) <= TOL
    assert np.array_equal(rho, rho.conj().T)


@pytest.mark.parametrize("n", [9, 10, 11])
def test_estimate_multipass_sampled(n):
    """Sizes with several later passes and many counts-pass tiles: sampled coefficients
    bit-exact, sampled rho entries against eq. (4) on the GPU coefficients."""
    print(f"[estimate sampled n={n}]", flush=True)
    shots = 300
    counts = _haar_counts(n, shots, 40 + n)
    coef, rho = L.estimate(_dev(counts), shots)
    coef, rho = coef.cpu().numpy(), rho.cpu().numpy()
    rng = np.random.default_rng(n)
    idx = np.concatenate([[0, 1, 2, 3, 4 ** n - 1], rng.integers(0, 4 ** n, 400)])
    np.testing.assert_array_equal(coef[idx], oracle.coefs(n, counts, shots, idx=idx))
    r = rng.integers(0, 2 ** n, 300)
    c = rng.integers(0, 2 ** n, 300)
    ref = oracle.rho(n, coef, r, c)
    assert np.max(np.abs(rho[r, c] - ref)) <= TOL
    assert np.array_equal(rho, rho.conj().T)
    assert abs(np.trace(rho) - 1) <= TOL


@pytest.mark.parametrize("n", [1, 5, 7, 10])
def test_signed_sums_bit_exact(n):
    print(f"[signed_sums n={n}]", flush=True)
    counts = _haar_counts(n, 500, 50 + n)
    rng = np.random.default_rng(n)
    bases = np.unique(np.concatenate([[0, 3 ** n - 1], rng.integers(0, 3 ** n, 20)]))
    S = L.signed_sums(_dev(counts), _dev(bases.astype(np.int64))).cpu().numpy()
    ms = np.arange(2 ** n) if n <= 7 else rng.integers(0, 2 ** n, 200)
    bb = np.repeat(bases, len(ms))
    mm = np.tile(ms, len(bases))
    ii = np.array([_walsh_coef_index(n, int(b), int(m)) for b, m in zip(bb, mm)])
    ref = oracle.basis_sums(n, counts, bb, ii)
    np.testing.assert_array_equal(S[:, ms].ravel(), ref)


@pytest.mark.parametrize("n", [6, 7, 9, 11])
def test_signed_sums_mfma_bit_exact(n):
    """lre_signed_sums through the int8-MFMA 64-outcome transform of the MFMA counts pass:
    equal to the plain sums and to the oracle; counts up to 65535 (both byte limbs)."""
    print(f"[signed_sums MFMA n={n}]", flush=True)
    rng = np.random.default_rng(90 + n)
    if n <= 9:
        counts = _haar_counts(n, 500, 60 + n)
        counts[:3] = rng.integers(0, 65536, size=(3, 2 ** n))          # full uint16 range
    else:
        counts = rng.integers(0, 13, size=(3 ** n, 2 ** n), dtype=np.uint16)
    bases = np.unique(np.concatenate([[0, 1, 2, 3 ** n - 1], rng.integers(0, 3 ** n, 24)]))
    c, b = _dev(counts), _dev(bases.astype(np.int64))
    S_m = L.signed_sums(c, b, flags=L.LRE_WHT_MFMA).cpu().numpy()
    S_p = L.signed_sums(c, b).cpu().numpy()
    np.testing.assert_array_equal(S_m, S_p)
    ms = np.arange(2 ** n) if n <= 7 else rng.integers(0, 2 ** n, 300)
    bb = np.repeat(bases, len(ms))
    mm = np.tile(ms, len(bases))
    ii = np.array([_walsh_coef_index(n, int(x), int(m)) for x, m in zip(bb, mm)])
    np.testing.assert_array_equal(S_m[:, ms].ravel(), oracle.basis_sums(n, counts, bb, ii))


def test_signed_sums_mfma_small_n_unsupported():
    counts = _dev(_haar_counts(5, 100, 7))
    with pytest.raises(L.LreError) as e:
        L.signed_sums(counts, _dev(np.array([0, 1], dtype=np.int64)), flags=L.LRE_WHT_MFMA)
    assert e.value.status == L.LRE_E_UNSUPPORTED


@pytest.mark.parametrize("n", [3, 8, 10])
def test_maximally_mixed_exact(n):
    """Equal counts: every non-identity coefficient is exactly 0 and rho = I / 2^n."""
    print(f"[maximally mixed n={n}]", flush=True)
    K = 5
    coef, rho = L.estimate(_dev(ti.maximally_mixed_counts(n, K)), K * 2 ** n)
    coef, rho = coef.cpu().numpy(), rho.cpu().numpy()
    assert coef[0] == 1.0 and np.all(coef[1:] == 0.0)
    assert np.array_equal(rho, np.eye(2 ** n) / 2 ** n)


@pytest.mark.parametrize("n,p_dep", [(4, 0.0), (7, 0.5), (9, 0.0)])
def test_ghz_exact(n, p_dep):
    print(f"[ghz n={n}]", flush=True)
    shots = 2 ** (n + 1)
    counts = ti.exact_counts(ti.ghz_probs(n, p_dep), shots)
    coef, rho = L.estimate(_dev(counts), shots)
    coef, rho = coef.cpu().numpy(), rho.cpu().numpy()
    np.testing.assert_array_equal(coef, refs.ghz_expectations(n, p_dep))
    assert np.max(np.abs(rho - refs.ghz_density(n, p_dep))) <= TOL


@pytest.mark.parametrize("n", [5, 7, 8, 9, 10, 11, 12])
def test_rho_fp32_is_rounded_fp64(n):
    """LRE_RHO_FP32 writes the binary64 entries rounded to complex64: every step-(ii)
    form (n <= 6 in LDS, the tiles for 7 <= n <= 10, the intermediate for n >= 11) gives
    exactly the complex128 result converted.  Uniform shots (paired Philox counts), so
    that the two calls' coefficients are the same exact integer quotients (per-basis
    binary64 sums can differ in the last bit between calls: LDS atomics from different
    waves land in run-dependent order)."""
    import tomo_inputs.gpu as tg
    print(f"[rho fp32 n={n}]", flush=True)
    counts, _ = tg.philox_counts(n, 0x1602_0860_4F + n, device=DEV, paired=True)
    shots = 12 << (n - 1)
    coef, rho64 = L.estimate(counts, shots)
    _, rho32 = L.estimate(counts, shots, flags=L.LRE_RHO_FP32)
    assert rho32.dtype == torch.complex64
    assert torch.equal(rho32, rho64.to(torch.complex64))
    assert (rho32.to(torch.complex128) - rho64).abs().max().item() < 1e-7


@pytest.mark.parametrize("n,flags", [(4, 0), (8, 0), (8, "mfma"), (10, 0), (12, "mfma")])
def test_estimate_graph_replay(n, flags):
    """lre_estimate enqueues kernels only, so a caller can capture one step into a HIP
    graph: every replay (outputs cleared before it, eager estimates of other counts and
    synchronisations between replays) equals the eager call bit for bit, and a data error
    raised inside a replay still reaches the flag word."""
    import tomo_inputs.gpu as tg
    print(f"[graph replay n={n} flags={flags}]", flush=True)
    fl = L.LRE_WHT_MFMA if flags == "mfma" else 0
    counts, _ = tg.philox_counts(n, 0x6A0 + n, device=DEV, paired=True)
    other, _ = tg.philox_counts(n, 0x6B0 + n, device=DEV, paired=True)
    shots = 12 << (n - 1)
    ref_coef, ref_rho = L.estimate(counts, shots, flags=fl)
    coef = torch.empty_like(ref_coef)
    rho = torch.empty_like(ref_rho)
    ws = torch.empty(max(L.workspace_bytes(n, shots, fl), 1), dtype=torch.uint8, device=DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        L.estimate(counts, shots, flags=fl, coef=coef, rho=rho, workspace=ws, check=False)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        L.estimate(counts, shots, flags=fl, coef=coef, rho=rho, workspace=ws, check=False)
    for k in range(3):
        coef.zero_()
        rho.zero_()
        g.replay()
        torch.cuda.synchronize()
        L.check_flags(DEV)
        assert torch.equal(coef, ref_coef), f"replay {k}: coefficients"
        assert torch.equal(rho, ref_rho), f"replay {k}: rho"
        oc, orho = L.estimate(other, shots, flags=fl)      # eager work between replays
        assert not torch.equal(oc, ref_coef)
        del oc, orho
    del g
    # a capture whose shot count disagrees with the rows: the replay sets the flag
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        L.estimate(counts, shots + 1, flags=fl, coef=coef, rho=rho, workspace=ws, check=False)
    g.replay()
    with pytest.raises(L.LreError) as e:
        L.check_flags(DEV)
    assert e.value.status == L.LRE_E_SHOTS
    del g
    coef2, _ = L.estimate(counts, shots, flags=fl)
    assert torch.equal(coef2, ref_coef)


@pytest.mark.parametrize("n", [11, 12])
def test_rho_real_tiles_full_rows(n):
    """Step (ii) at 11 and 12 qubits (real-arithmetic tiles, no intermediate): whole rows
    of rho -- every column pattern x, so every tile -- against eq. (4) on the GPU's
    coefficients, rho exactly Hermitian with unit trace, for complex128 and complex64."""
    import tomo_inputs.gpu as tg
    print(f"[rho real tiles n={n}]", flush=True)
    counts, _ = tg.philox_counts(n, 0x7A11 + n, device=DEV, paired=True)
    shots = 12 << (n - 1)
    coef, rho = L.estimate(counts, shots)
    e = coef.cpu().numpy()
    d = 2 ** n
    rows = np.array([0, d - 1] + list(np.random.default_rng(n).integers(0, d, 2)))
    for r in rows:
        got = rho[int(r)].cpu().numpy()
        ref = oracle.rho(n, e, np.full(d, r), np.arange(d))
        assert np.max(np.abs(got - ref)) <= TOL, f"row {r}"
    assert bool(torch.equal(rho, rho.conj().transpose(0, 1).contiguous()))
    assert abs(torch.diagonal(rho).sum().item() - 1) <= TOL
    _, rho32 = L.estimate(counts, shots, flags=L.LRE_RHO_FP32)
    assert torch.equal(rho32, rho.to(torch.complex64))


def test_no_rho_flag():
    counts = _haar_counts(6, 100, 61)
    coef, rho = L.estimate(_dev(counts), 100, flags=L.LRE_NO_RHO)
    assert rho is None
    np.testing.assert_array_equal(coef.cpu().numpy(), oracle.coefs(6, counts, 100))


def test_error_flags():
    counts = ti.maximally_mixed_counts(5, 2)
    with pytest.raises(L.LreError) as e:
        L.estimate(_dev(counts), 63)                       # rows sum to 64
    assert e.value.status == L.LRE_E_SHOTS
    bad = counts.copy()
    bad[7] = 0
    with pytest.raises(L.LreError) as e:
        L.estimate(_dev(bad), 0)                           # empty basis, per-basis mode
    assert e.value.status == L.LRE_E_EMPTY_BASIS
    nb = _dev(np.full(3 ** 5, 64, dtype=np.int32))
    nb[3] = 65
    with pytest.raises(L.LreError) as e:
        L.estimate(_dev(counts), 0, n_per_basis=nb)        # declared total differs
    assert e.value.status == L.LRE_E_SHOTS
    # after an error the flag word is clear again
    coef, _ = L.estimate(_dev(counts), 64)
    assert coef[0].item() == 1.0


def test_host_side_argument_errors():
    counts = _dev(ti.maximally_mixed_counts(3, 1))
    coef = torch.empty(64, dtype=torch.float64, device=DEV)
    ctx = L.context(0)
    lib = L.lib()
    import ctypes
    P = ctypes.c_void_p
    st = torch.cuda.current_stream().cuda_stream
    ws = torch.empty(L.workspace_bytes(3, 8), dtype=torch.uint8, device=DEV)
    # misaligned counts
    assert lib.lre_estimate(P(ctx), 3, P(counts.data_ptr() + 2), 8, None, P(coef.data_ptr()), None,
                            P(ws.data_ptr()), ws.numel(), L.LRE_NO_RHO, P(st)) == L.LRE_E_ARG
    # workspace too small
    assert lib.lre_estimate(P(ctx), 3, P(counts.data_ptr()), 8, None, P(coef.data_ptr()), None,
                            P(ws.data_ptr()), 16, L.LRE_NO_RHO, P(st)) == L.LRE_E_WORKSPACE
    # n out of range
    assert lib.lre_estimate(P(ctx), 15, P(counts.data_ptr()), 8, None, P(coef.data_ptr()), None,
                            P(ws.data_ptr()), ws.numel(), L.LRE_NO_RHO, P(st)) == L.LRE_E_ARG
    # rho requested but NULL
    assert lib.lre_estimate(P(ctx), 3, P(counts.data_ptr()), 8, None, P(coef.data_ptr()), None,
                            P(ws.data_ptr()), ws.numel(), 0, P(st)) == L.LRE_E_ARG


def test_repeatable_and_linear():
    """Deterministic output, and linearity of the integer sums in the counts."""
    n = 9
    a = _haar_counts(n, 200, 70)
    b = _haar_counts(n, 200, 71)
    Ta = L.pauli_sums(_dev(a), 200)
    Ta2 = L.pauli_sums(_dev(a), 200)
    Tb = L.pauli_sums(_dev(b), 200)
    Tab = L.pauli_sums(_dev((a + b).astype(np.uint16)), 400)
    assert torch.equal(Ta, Ta2)
    assert torch.equal(Ta + Tb, Tab)


# ---- int8-MFMA counts pass: same bars, and bit-identical to the plain kernel ----

@pytest.mark.parametrize("n", [7, 8, 9, 10])
def test_mfma_pauli_sums_bit_exact(n):
    print(f"[mfma pauli_sums n={n}]", flush=True)
    shots = 1000 if n < 9 else 300
    counts = _haar_counts(n, shots, 80 + n)
    c = _dev(counts)
    T_m = L.pauli_sums(c, shots, flags=L.LRE_WHT_MFMA)
    T_p = L.pauli_sums(c, shots)
    assert torch.equal(T_m, T_p)
    T_m = T_m.cpu().numpy()
    if n <= 8:
        np.testing.assert_array_equal(T_m, oracle.pauli_sums(n, counts))
    else:
        idx = np.random.default_rng(n).integers(0, 4 ** n, 2000)
        np.testing.assert_array_equal(T_m[idx], oracle.pauli_sums(n, counts, idx))


def test_mfma_full_uint16_range():
    """Counts up to 65535 (both byte limbs used, binary64 partial sums): every row a
    permutation of one vector, so all rows share one total."""
    n = 7
    rng = np.random.default_rng(90)
    v = rng.integers(0, 65536, size=2 ** n).astype(np.uint16)
    v[:4] = [65535, 65535, 0, 32768]
    counts = np.stack([rng.permutation(v) for _ in range(3 ** n)])
    shots = int(v.astype(np.int64).sum())
    c = _dev(counts)
    T_m = L.pauli_sums(c, shots, flags=L.LRE_WHT_MFMA)
    assert torch.equal(T_m, L.pauli_sums(c, shots))
    np.testing.assert_array_equal(T_m.cpu().numpy(), oracle.pauli_sums(n, counts))
    coef, _ = L.estimate(c, shots, flags=L.LRE_WHT_MFMA | L.LRE_NO_RHO)
    np.testing.assert_array_equal(coef.cpu().numpy(), oracle.coefs(n, counts, shots))


@pytest.mark.parametrize("n", [7, 8])
def test_mfma_estimate_uniform_bit_exact(n):
    print(f"[mfma estimate uniform n={n}]", flush=True)
    shots = 2000
    counts = _haar_counts(n, shots, 100 + n)
    coef, rho = L.estimate(_dev(counts), shots, flags=L.LRE_WHT_MFMA)
    coef, rho = coef.cpu().numpy(), rho.cpu().numpy()
    e_ref = oracle.coefs(n, counts, shots)
    np.testing.assert_array_equal(coef, e_ref)
    assert np.max(np.abs(rho - oracle.rho(n, e_ref))) <= TOL


@pytest.mark.parametrize("n,nb_given", [(7, True), (8, False), (9, True)])
def test_mfma_estimate_per_basis(n, nb_given):
    print(f"[mfma estimate per-basis n={n}]", flush=True)
    rng = np.random.default_rng(110 + n)
    shots = rng.integers(100, 3000, size=3 ** n)
    counts = ti.multinomial_counts(ti.born_probs_pure(n, ti.haar_state(n, rng)), shots, rng)
    nb = _dev(counts.sum(axis=1).astype(np.int32)) if nb_given else None
    coef, _ = L.estimate(_dev(counts), 0, n_per_basis=nb, flags=L.LRE_WHT_MFMA | L.LRE_NO_RHO)
    coef = coef.cpu().numpy()
    coef_p, _ = L.estimate(_dev(counts), 0, n_per_basis=nb, flags=L.LRE_NO_RHO)
    assert np.max(np.abs(coef - coef_p.cpu().numpy())) <= TOL
    if n <= 8:
        assert np.max(np.abs(coef - oracle.coefs(n, counts, 0))) <= TOL
    else:
        idx = np.random.default_rng(n).integers(0, 4 ** n, 500)
        assert np.max(np.abs(coef[idx] - oracle.coefs(n, counts, 0, idx=idx))) <= TOL
    assert abs(coef[0] - 1.0) <= TOL    # rounded reciprocal of N_b: trace 1 up to rounding


def test_mfma_error_flags():
    counts = ti.maximally_mixed_counts(7, 2)
    with pytest.raises(L.LreError) as e:
        L.estimate(_dev(counts), 255, flags=L.LRE_WHT_MFMA)
    assert e.value.status == L.LRE_E_SHOTS
    coef, _ = L.estimate(_dev(counts), 256, flags=L.LRE_WHT_MFMA)
    c = coef.cpu().numpy()
    assert c[0] == 1.0 and np.all(c[1:] == 0.0)
