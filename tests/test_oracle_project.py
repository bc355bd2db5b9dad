"""Pins of the step-(iii) oracle (oracle/project.py) against facts fixed by the
mathematics, none of them the oracle compared with itself:

* a spectrum truncated by hand (the worked case below);
* the Euclidean projection onto the probability simplex computed by a different
  method (sort and threshold: keep the largest entries u_1 >= ... >= u_k with
  u_k - (sum_{j<=k} u_j - 1)/k > 0 and subtract that common shift), which the closest
  density matrix must reproduce on the spectrum;
* idempotence on physical input, and the closest-point property against random
  density matrices.
"""
import numpy as np
import pytest

from oracle import project as P


def _simplex_sort_threshold(u):
    s = np.sort(u)[::-1]
    cs = np.cumsum(s)
    k = np.arange(1, u.size + 1)
    ok = s - (cs - 1.0) / k > 0
    kk = k[ok][-1]
    theta = (cs[kk - 1] - 1.0) / kk
    return np.maximum(u - theta, 0.0)


def _random_density(d, rank, rng):
    g = rng.normal(size=(d, rank)) + 1j * rng.normal(size=(d, rank))
    r = g @ g.conj().T
    return r / np.trace(r).real


def _random_trace1_hermitian(d, rng, spread=0.3):
    h = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    h = (h + h.conj().T) / 2
    rho = _random_density(d, 2, rng)
    mu = rho + spread / d * (h - np.trace(h).real / d * np.eye(d))
    return mu


def test_hand_worked_spectrum():
    # m = (0.7, 0.45, -0.05, -0.1): -0.1 + 0/4 < 0 -> 0, a = -0.1; -0.05 - 0.1/3 < 0 -> 0,
    # a = -0.15; 0.45 - 0.15/2 = 0.375 >= 0 -> keep two, each lowered by 0.075.
    lam = P.truncate_spectrum(np.array([0.7, 0.45, -0.05, -0.1]))
    np.testing.assert_allclose(lam, [0.625, 0.375, 0.0, 0.0], atol=1e-15)


@pytest.mark.parametrize("seed", range(20))
def test_spectrum_matches_sort_threshold_projection(seed):
    rng = np.random.default_rng(seed)
    d = int(rng.choice([2, 4, 8, 16, 64]))
    u = rng.normal(size=d) * rng.uniform(0.01, 0.5)
    u = u - u.mean() + 1.0 / d                      # trace 1
    np.testing.assert_allclose(P.truncate_spectrum(u), _simplex_sort_threshold(u), atol=1e-14)


@pytest.mark.parametrize("d", [2, 4, 16])
def test_physical_input_is_unchanged(d):
    rng = np.random.default_rng(d)
    rho = _random_density(d, max(1, d // 2), rng)
    out, m, lam = P.project(rho)
    assert np.all(m > -1e-14)
    assert np.max(np.abs(out - rho)) <= 1e-13


@pytest.mark.parametrize("d", [4, 16, 64])
def test_result_is_the_closest_density_matrix(d):
    rng = np.random.default_rng(100 + d)
    mu = _random_trace1_hermitian(d, rng, spread=2.0)
    rho, m, lam = P.project(mu)
    assert m[0] < 0                                 # the case is not trivial
    ev = np.linalg.eigvalsh(rho)
    assert ev.min() > -1e-13 and abs(np.trace(rho).real - 1) < 1e-13
    assert np.max(np.abs(rho - rho.conj().T)) < 1e-14
    best = np.linalg.norm(mu - rho)
    for _ in range(200):
        sigma = _random_density(d, int(rng.integers(1, d + 1)), rng)
        assert np.linalg.norm(mu - sigma) >= best - 1e-12
