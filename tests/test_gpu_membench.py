"""Streaming diagnostics (lre_stream_read / lre_stream_copy): the copy is exact on a
ragged size (not a multiple of the block range) and the read leaves its sink alone."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1602_08604_amd import lre as L  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("n", [4, 1000, (1 << 22) + 12])
def test_stream_copy_and_read(n):
    print(f"[stream diagnostics n={n}]", flush=True)
    g = torch.Generator(device=DEV).manual_seed(n)
    src = torch.randint(0, 2 ** 31 - 1, (n,), dtype=torch.int32, device=DEV, generator=g)
    dst = torch.zeros_like(src)
    L.stream_copy(src, dst)
    sink = torch.zeros(1, dtype=torch.int32, device=DEV)
    L.stream_read(src, sink)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    assert int(sink.item()) in (0, 0x9E3779B9 - 2 ** 32)


@pytest.mark.parametrize("kind", ["valu_i32", "mfma_i8"])
def test_peak_rate_diagnostics(kind):
    """The compute-rate diagnostics run, report their operation count and leave the sink
    alone; bad arguments are refused."""
    print(f"[peak {kind}]", flush=True)
    sink = torch.zeros(1, dtype=torch.int32, device=DEV)
    ops = L.peak_rate(kind, 3, sink)
    torch.cuda.synchronize()
    assert ops > 0 and int(sink.item()) == 0
    with pytest.raises(L.LreError) as e:
        L.peak_rate(kind, 0, sink)
    assert e.value.status == L.LRE_E_ARG
