"""Batched estimation (lre_batch_*): every instance equals its single-instance
lre_estimate result bit for bit and the oracle to the usual bars; work-list shapes,
graph capture and replay, the autotuner, FP32 rho and the error paths."""
import numpy as np
import pytest

import oracle
import tomo_inputs as ti

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1602_08604_amd import lre as L  # noqa: E402

DEV = "cuda:0"
TOL = 1e-12


def _instances(seed, ns):
    """Haar-state multinomial counts on the device, one seed per instance."""
    import tomo_inputs.gpu as tg
    rng = np.random.default_rng(seed)
    shots = [int(x) for x in rng.integers(100, 10_001, size=len(ns))]
    counts = [tg.haar_multinomial_counts(int(n), s, seed * 1000 + j, device=DEV)
              for j, (n, s) in enumerate(zip(ns, shots))]
    return counts, shots


def _single(c, s, flags=0):
    coef, rho = L.estimate(c, s, flags=flags)
    return coef, rho


def _check_against_single(b, flags=0):
    for j, (c, s) in enumerate(zip(b.counts, b.shots)):
        coef, rho = _single(c, s, flags)
        assert torch.equal(b.coefs[j], coef), f"instance {j} (n={b.n[j]}) coef differs"
        if not flags & L.LRE_NO_RHO:
            assert torch.equal(b.rhos[j], rho), f"instance {j} (n={b.n[j]}) rho differs"


def test_batch_matches_single_and_oracle():
    print("[batch: n = 1..9 mixed]", flush=True)
    ns = list(range(1, 10)) + [9, 8, 7, 3, 6, 9, 2, 8]
    counts, shots = _instances(11, ns)
    b = L.Batch(counts, shots)
    b.run(check=True)
    _check_against_single(b)
    rng = np.random.default_rng(3)
    for j, n in enumerate(b.n):
        host = counts[j].cpu().numpy()
        e = b.coefs[j].cpu().numpy()
        if n <= 7:
            np.testing.assert_array_equal(e, oracle.coefs(n, host, shots[j]))
            mu = b.rhos[j].cpu().numpy()
            assert np.max(np.abs(mu - oracle.rho(n, e))) <= TOL
        else:
            idx = np.concatenate([[0, 4 ** n - 1], rng.integers(0, 4 ** n, 300)])
            np.testing.assert_array_equal(e[idx], oracle.coefs(n, host, shots[j], idx=idx))
            r = rng.integers(0, 2 ** n, 200)
            c = rng.integers(0, 2 ** n, 200)
            mu = b.rhos[j][torch.from_numpy(r).to(DEV), torch.from_numpy(c).to(DEV)].cpu().numpy()
            assert np.max(np.abs(mu - oracle.rho(n, e, r, c))) <= TOL
    b.close()


@pytest.mark.parametrize("tiles", [(1, 1, 432, 1, 0), (2, 4, 432 * 16, 16, 1), (1, 3, 432 * 5, 7, 1),
                                   (2, 1, 432, 8, 0)])
def test_batch_tile_shapes(tiles):
    print(f"[batch tiles {tiles}]", flush=True)
    counts, shots = _instances(12, [9, 4, 8, 7, 1, 9, 6, 5])
    b = L.Batch(counts, shots)
    b.set_tiles(*tiles)
    b.run(check=True)
    _check_against_single(b)
    b.close()


def test_batch_no_rho_and_fp32():
    print("[batch NO_RHO / RHO_FP32]", flush=True)
    counts, shots = _instances(13, [9, 8, 5, 7, 3])
    b = L.Batch(counts, shots, flags=L.LRE_NO_RHO)
    b.run(check=True)
    _check_against_single(b, L.LRE_NO_RHO)
    b.close()
    b32 = L.Batch(counts, shots, flags=L.LRE_RHO_FP32)
    b32.run(check=True)
    _check_against_single(b32, L.LRE_RHO_FP32)
    b64 = L.Batch(counts, shots)
    b64.run(check=True)
    worst = 0.0
    for r32, r64 in zip(b32.rhos, b64.rhos):
        worst = max(worst, (r32.to(torch.complex128) - r64).abs().max().item())
    print(f"max |rho_fp32 - rho_fp64| = {worst:.3e}")
    assert worst < 1e-7


def test_batch_graph_capture_replay():
    """One captured launch replayed several times, with eager work between replays."""
    print("[batch graph capture]", flush=True)
    counts, shots = _instances(14, [9, 6, 8, 2, 7])
    b = L.Batch(counts, shots)
    b.run(check=True)
    want_c = [c.clone() for c in b.coefs]
    want_r = [r.clone() for r in b.rhos]
    b.workspace()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()                       # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(3):
        for c in b.coefs:
            c.zero_()
        for r in b.rhos:
            r.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        L.check_flags(DEV)
        for j in range(len(counts)):
            assert torch.equal(b.coefs[j], want_c[j]), f"replay {rep}: coef {j}"
            assert torch.equal(b.rhos[j], want_r[j]), f"replay {rep}: rho {j}"
    b.close()


def test_batch_tune_keeps_results():
    print("[batch tune]", flush=True)
    counts, shots = _instances(15, [9, 9, 8, 7, 5, 3])
    b = L.Batch(counts, shots)
    ms = b.tune(reps=2)
    print(f"tuned: {b.tiles} {ms:.3f} ms")
    assert ms > 0
    b.run(check=True)
    _check_against_single(b)
    b.close()


def test_batch_errors():
    print("[batch errors]", flush=True)
    counts, shots = _instances(16, [4, 7])
    with pytest.raises(L.LreError) as e:
        L.Batch(counts, [shots[0], 0])
    assert e.value.status == L.LRE_E_UNSUPPORTED
    big = torch.zeros((3 ** 10, 2 ** 10), dtype=torch.uint16, device=DEV)
    with pytest.raises(L.LreError) as e:
        L.Batch([big], [1])
    assert e.value.status == L.LRE_E_UNSUPPORTED
    del big
    with pytest.raises(L.LreError) as e:
        L.Batch([counts[0]], [2 ** 31 // 81 + 1])          # 3^n * shots beyond int32
    assert e.value.status == L.LRE_E_ARG
    # a basis that does not sum to the declared shots is flagged, the other instance is fine
    bad = counts[1].to(torch.int32)
    bad[5, 0] += 1
    bad = bad.to(torch.uint16)
    b = L.Batch([counts[0], bad], shots)
    b.run()
    with pytest.raises(L.LreError) as e:
        L.check_flags(DEV)
    assert e.value.status == L.LRE_E_SHOTS
    coef, _ = _single(counts[0], shots[0])
    assert torch.equal(b.coefs[0], coef)
    b.close()
