"""The on-device Philox generator equals its numpy twin bit for bit."""
import numpy as np
import pytest

import tomo_inputs as ti

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


@pytest.mark.parametrize("n,b0,nrows", [(1, 0, 3), (2, 0, 9), (5, 10, 50), (10, 1000, 64), (14, 4782900, 69)])
def test_philox_counts_match_twin(n, b0, nrows):
    from tomo_inputs import gpu
    seed = 0x1602_0860_4 + n
    c, nb = gpu.philox_counts(n, seed, b0, nrows)
    c = c.cpu().numpy()
    ref = ti.philox_counts_rows(n, seed, np.arange(b0, b0 + nrows))
    np.testing.assert_array_equal(c, ref)
    np.testing.assert_array_equal(nb.cpu().numpy(), ref.sum(axis=1).astype(np.int64))
    c, nb = gpu.philox_counts(n, seed, b0, nrows, paired=True)
    ref, rnb = ti.philox_counts_rows_fast(n, seed, np.arange(b0, b0 + nrows), paired=True)
    np.testing.assert_array_equal(c.cpu().numpy(), ref)
    np.testing.assert_array_equal(nb.cpu().numpy(), rnb.astype(np.int64))
