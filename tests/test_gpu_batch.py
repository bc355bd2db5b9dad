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
                                   (2, 1, 432, 8, 0), (1, 4, 432 * 16, 1, 0, 1), (2, 1, 432, 1, 0, 1),
                                   (1, 2, 432 * 4, 2, 1, 1)])
def test_batch_tile_shapes(tiles):
    print(f"[batch tiles {tiles}]", flush=True)
    counts, shots = _instances(12, [9, 4, 8, 7, 1, 9, 6, 5])
    b = L.Batch(counts, shots)
    b.set_tiles(*tiles)
    b.run(check=True)
    _check_against_single(b)
    b.close()


@pytest.mark.parametrize("ns", [[3, 5, 7, 1], [8], [9, 9], [7, 8]])
def test_batch_staged_edge_sets(ns):
    """The staged form with no later stage at all (every instance of at most 7 qubits),
    with only one size of larger instance, and mixed."""
    print(f"[batch staged {ns}]", flush=True)
    counts, shots = _instances(21, ns)
    b = L.Batch(counts, shots)
    b.set_tiles(1, 4, 432 * 16, 1, 0, 1)
    b.run(check=True)
    _check_against_single(b)
    b.close()


@pytest.mark.parametrize("staged", [0, 1])
def test_batch_no_rho_and_fp32(staged):
    print(f"[batch NO_RHO / RHO_FP32, staged={staged}]", flush=True)
    counts, shots = _instances(13, [9, 8, 5, 7, 3])
    b = L.Batch(counts, shots, flags=L.LRE_NO_RHO)
    b.set_tiles(1, 4, 432 * 16, 1, 0, staged)
    b.run(check=True)
    _check_against_single(b, L.LRE_NO_RHO)
    b.close()
    b32 = L.Batch(counts, shots, flags=L.LRE_RHO_FP32)
    b32.set_tiles(1, 4, 432 * 16, 1, 0, staged)
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


@pytest.mark.parametrize("captured", [(1, 4, 432 * 16, 1, 0, 0), (1, 4, 432 * 16, 1, 0, 1)])
def test_batch_graph_survives_retune(captured):
    """A launch captured before lre_batch_set_tiles replays the new work list (the list
    keeps its address and the kernels read the item count and the staged flag from
    device memory), between the staged and unstaged forms too."""
    print(f"[batch graph + retune, captured with {captured}]", flush=True)
    counts, shots = _instances(17, [9, 8, 9, 7, 4, 8])
    b = L.Batch(counts, shots)
    b.set_tiles(*captured)
    b.run(check=True)
    want_c = [c.clone() for c in b.coefs]
    want_r = [r.clone() for r in b.rhos]
    b.workspace()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    items0 = b.tiles["items"]
    for shape in ((1, 1, 432, 4, 1), (1, 2, 432 * 4, 2, 0, 1), (1, 2, 432 * 4, 2, 0), (2, 1, 432, 1, 0, 1),
                  captured):
        b.set_tiles(*shape)
        print(f"  retuned to {b.tiles} (captured with {items0} items)", flush=True)
        for c in b.coefs:
            c.zero_()
        for r in b.rhos:
            r.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        L.check_flags(DEV)
        for j in range(len(counts)):
            assert torch.equal(b.coefs[j], want_c[j]), f"{shape}: coef {j}"
            assert torch.equal(b.rhos[j], want_r[j]), f"{shape}: rho {j}"
    b.close()


def test_batch_per_basis():
    """Per-basis totals inside a batch (shots = 0): N_b given or taken from the rows,
    against the single-instance per-basis estimate (1e-12) and the oracle (1e-12),
    mixed with uniform-shot instances (those stay bit-identical)."""
    print("[batch per-basis]", flush=True)
    import tomo_inputs.gpu as tg
    ns = [9, 3, 8, 7, 5, 9, 1, 8]
    rng = np.random.default_rng(18)
    counts, nbs, shots = [], [], []
    for j, n in enumerate(ns):
        s = int(rng.integers(100, 3000))
        c = tg.haar_multinomial_counts(n, s, 18000 + j, device=DEV).to(torch.int32)
        if j % 2 == 0:              # uneven totals: add 0..5 counts to each basis's first outcome
            c[:, 0] += torch.from_numpy(rng.integers(0, 6, size=3 ** n).astype(np.int32)).to(DEV)
        c = c.to(torch.uint16)
        counts.append(c)
        nb = c.to(torch.int64).sum(dim=1).to(torch.int32)
        if j % 2 == 0:
            shots.append(0)
            nbs.append(nb if j % 4 == 0 else None)
        else:
            shots.append(s)
            nbs.append(None)
    for flags in (0, L.LRE_RHO_FP32):
        b = L.Batch(counts, shots, flags=flags, n_per_basis=nbs)
        b.run(check=True)
        for j, n in enumerate(ns):
            coef, rho = L.estimate(counts[j], shots[j], n_per_basis=nbs[j], flags=flags)
            if shots[j]:
                assert torch.equal(b.coefs[j], coef), f"instance {j}"
                assert torch.equal(b.rhos[j], rho), f"instance {j}"
                continue
            assert (b.coefs[j] - coef).abs().max().item() <= TOL, f"instance {j}"
            tol_r = TOL if flags == 0 else 1e-6
            assert (b.rhos[j].to(torch.complex128) - rho.to(torch.complex128)).abs().max().item() <= tol_r
            host = counts[j].cpu().numpy()
            e = b.coefs[j].cpu().numpy()
            idx = np.arange(4 ** n) if n <= 6 else np.concatenate(
                [[0, 4 ** n - 1], np.random.default_rng(j).integers(0, 4 ** n, 300)])
            ref = oracle.coefs(n, host, 0, idx=idx)
            assert np.max(np.abs(e[idx] - ref)) <= TOL, f"instance {j}"
        for shape in ("tuned", (1, 2, 432 * 16, 1, 0, 1)):
            if shape == "tuned":
                b.tune(reps=1)
            else:
                b.set_tiles(*shape)
            b.run(check=True)
            for j in range(len(ns)):
                coef, rho = L.estimate(counts[j], shots[j], n_per_basis=nbs[j], flags=flags)
                assert (b.coefs[j] - coef).abs().max().item() <= TOL, f"{shape}: instance {j}"
                tol_r = TOL if flags == 0 else 1e-6
                assert (b.rhos[j].to(torch.complex128) - rho.to(torch.complex128)).abs().max().item() <= tol_r
        b.close()


def test_batch_per_basis_errors():
    """Per-basis data errors in a batch: declared totals that differ from the row sums
    (LRE_E_SHOTS) and an empty basis (LRE_E_EMPTY_BASIS)."""
    print("[batch per-basis errors]", flush=True)
    counts, shots = _instances(19, [8, 5])
    nb = counts[0].to(torch.int64).sum(dim=1).to(torch.int32)
    nb[7] += 1
    b = L.Batch(counts, [0, 0], n_per_basis=[nb, None])
    b.run()
    with pytest.raises(L.LreError) as e:
        L.check_flags(DEV)
    assert e.value.status == L.LRE_E_SHOTS
    b.close()
    empty = counts[1].to(torch.int32)
    empty[4] = 0
    empty = empty.to(torch.uint16)
    b = L.Batch([counts[0], empty], [0, 0])
    b.run()
    with pytest.raises(L.LreError) as e:
        L.check_flags(DEV)
    assert e.value.status == L.LRE_E_EMPTY_BASIS
    b.close()
