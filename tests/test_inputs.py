"""Pins of the seeded input generators (shared by the oracle side and the GPU side)."""
import numpy as np
import pytest

import tomo_inputs as ti
from tests import refs


def test_philox_known_answers():
    """Known-answer vectors published with the Random123 reference implementation of
    Philox4x32-10 (Salmon et al., SC'11)."""
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = ti.philox4x32_10(*ctr, *key)
        assert tuple(int(v) for v in got) == want


def test_philox_counts_range_and_uniformity():
    c = ti.philox_counts_rows(10, 20240, np.arange(200))
    assert c.dtype == np.uint16 and c.shape == (200, 1024)
    assert c.min() == 0 and c.max() == 12
    freq = np.bincount(c.ravel(), minlength=13) / c.size
    assert np.max(np.abs(freq - 1 / 13)) < 0.005


@pytest.mark.parametrize("n", [1, 2, 3])
def test_born_probabilities_match_explicit_projectors(n):
    rng = np.random.default_rng(50 + n)
    psi = ti.haar_state(n, rng)
    p = ti.born_probs_pure(n, psi)
    np.testing.assert_allclose(p, refs.born_from_projectors(n, np.outer(psi, psi.conj())),
                               rtol=0, atol=1e-14)
    G = ti.ginibre_factor(n, 3, rng)
    np.testing.assert_allclose(ti.born_probs_mixed(n, G),
                               refs.born_from_projectors(n, G @ G.conj().T), rtol=0, atol=1e-14)


@pytest.mark.parametrize("n,p_dep", [(2, 0.0), (3, 0.05)])
def test_ghz_probabilities(n, p_dep):
    p = ti.ghz_probs(n, p_dep)
    np.testing.assert_allclose(p, refs.born_from_projectors(n, refs.ghz_density(n, p_dep)),
                               rtol=0, atol=1e-14)
    lo = ti.ghz_probs(n, p_dep, 2, 7)
    np.testing.assert_array_equal(lo, p[2:7])
    with pytest.raises(ValueError):
        ti.ghz_probs(n, p_dep, 0, 3 ** n + 1)


def test_multinomial_rows_sum_to_shots():
    rng = np.random.default_rng(3)
    p = ti.born_probs_pure(4, ti.haar_state(4, rng))
    shots = rng.integers(100, 10_000, size=81)
    c = ti.multinomial_counts(p, shots, rng)
    assert np.array_equal(c.sum(axis=1), shots)


def test_philox_c_twin_matches_numpy_twin():
    bases = np.array([0, 1, 2, 12345, 4782968])
    c, nb = ti.philox_counts_rows_fast(14, 987654321, bases)
    ref = ti.philox_counts_rows(14, 987654321, bases)
    np.testing.assert_array_equal(c, ref)
    np.testing.assert_array_equal(nb, ref.sum(axis=1))
    for n in (1, 3, 14):                       # paired rows: odd outcome = 12 - even one
        b = bases[bases < 3 ** n]
        c, nb = ti.philox_counts_rows_fast(n, 987654321, b, paired=True)
        ref = ti.philox_counts_rows(n, 987654321, b).astype(np.int64)
        np.testing.assert_array_equal(c[:, 0::2], ref[:, 0::2])
        np.testing.assert_array_equal(c[:, 1::2], 12 - ref[:, 0::2])
        assert np.all(nb == 12 << (n - 1))


def test_device_rotated_amplitudes_match_numpy():
    """The torch mode-product form of the Born amplitudes equals the numpy one (CPU)."""
    torch = pytest.importorskip("torch")
    import tomo_inputs.gpu as tg
    rng = np.random.default_rng(77)
    for n in (1, 3, 5):
        psi = ti.haar_state(n, rng)
        a = ti.rotated_amplitudes(n, psi)
        b = tg.rotated_amplitudes(n, torch.from_numpy(psi)).numpy()
        np.testing.assert_allclose(b, a, rtol=0, atol=1e-14)
