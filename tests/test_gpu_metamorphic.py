"""Metamorphic properties of the HIP path (through the C ABI).

* Qubit relabelling: permuting the qubits of the measurement record (the basis letters
  and the outcome bits of every setting alike) permutes the Pauli letters of every
  coefficient in the same way.  With uniform shots the coefficients are exact integer
  quotients, so the permuted run equals the permuted coefficients bit for bit, on the
  plain and on the int8-MFMA Walsh paths.
* Outcome flip: exchanging the two outcomes of qubit k in every setting (s -> s ^ bit k)
  negates exactly the coefficients whose letter at k is X, Y or Z (the one-qubit Gamma
  vectors of Sec. III change sign in their non-identity entry), and leaves the others
  unchanged.  With uniform shots (exact integer sums) this holds bit for bit.  The
  per-basis branch sums binary64 terms through LDS atomics whose order is not fixed,
  so there the relation is checked to 1e-12, the bar for per-basis coefficients.
* Outcome flip on mu: eq. (4) is linear in the coefficients, and negating the X, Y, Z
  letters of qubit k maps a one-qubit operator M to Tr(M) I - M; the flipped run's mu is
  that map applied to qubit k of mu, to rounding (checked to 1e-12, the bar for mu).
"""
import numpy as np
import pytest

import tomo_inputs as ti

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


def _relabel_counts(n, counts, perm):
    """New qubit q (0 = most significant, the paper's qubit 1) is old qubit perm[q]."""
    t = counts.reshape((3,) * n + (2,) * n)
    t = np.transpose(t, list(perm) + [n + p for p in perm])
    return np.ascontiguousarray(t.reshape(3 ** n, 2 ** n))


def _relabel_coef(n, coef, perm):
    t = coef.reshape((4,) * n)
    return np.ascontiguousarray(np.transpose(t, list(perm)).reshape(4 ** n))


def _flip_counts(n, counts, q):
    """Exchange the outcomes of qubit q (0 = most significant) in every setting."""
    bit = 1 << (n - 1 - q)
    s = np.arange(2 ** n)
    return np.ascontiguousarray(counts[:, s ^ bit])


def _nonidentity_at(n, q):
    i = np.arange(4 ** n)
    return ((i >> (2 * (n - 1 - q))) & 3) != 0


@pytest.mark.parametrize("n,flags", [(5, 0), (7, 0), (8, L.LRE_WHT_MFMA), (9, 0)])
def test_qubit_relabelling_permutes_coefficients(n, flags):
    print(f"[relabel n={n} flags={flags}]", flush=True)
    shots = 600
    counts = _haar_counts(n, shots, 300 + n)
    perm = np.random.default_rng(n).permutation(n)
    e, _ = L.estimate(_dev(counts), shots, flags=flags | L.LRE_NO_RHO)
    e2, _ = L.estimate(_dev(_relabel_counts(n, counts, perm)), shots, flags=flags | L.LRE_NO_RHO)
    np.testing.assert_array_equal(e2.cpu().numpy(), _relabel_coef(n, e.cpu().numpy(), perm))


@pytest.mark.parametrize("n,q,flags", [(4, 0, 0), (7, 6, 0), (8, 2, L.LRE_WHT_MFMA), (9, 4, 0)])
def test_outcome_flip_negates_uniform(n, q, flags):
    print(f"[flip uniform n={n} q={q} flags={flags}]", flush=True)
    shots = 500
    counts = _haar_counts(n, shots, 400 + n)
    e, mu = L.estimate(_dev(counts), shots, flags=flags)
    e2, mu2 = L.estimate(_dev(_flip_counts(n, counts, q)), shots, flags=flags)
    e, e2 = e.cpu().numpy(), e2.cpu().numpy()
    sel = _nonidentity_at(n, q)
    np.testing.assert_array_equal(e2[sel], -e[sel])
    np.testing.assert_array_equal(e2[~sel], e[~sel])
    # mu' = (Tr_q(.) I - .) on qubit q: entries (r_q, c_q) of the qubit-q block
    a, b = 1 << q, 1 << (n - 1 - q)
    m = mu.reshape(a, 2, b, a, 2, b)
    tr = m[:, 0, :, :, 0, :] + m[:, 1, :, :, 1, :]
    ref = -m.clone()
    ref[:, 0, :, :, 0, :] += tr
    ref[:, 1, :, :, 1, :] += tr
    assert (mu2 - ref.reshape(mu.shape)).abs().max().item() <= TOL


@pytest.mark.parametrize("n,q,flags", [(6, 1, 0), (8, 7, 0), (9, 3, L.LRE_WHT_MFMA)])
def test_outcome_flip_negates_per_basis(n, q, flags):
    print(f"[flip per-basis n={n} q={q} flags={flags}]", flush=True)
    rng = np.random.default_rng(500 + n)
    shots = rng.integers(100, 3000, size=3 ** n)
    counts = ti.multinomial_counts(ti.born_probs_pure(n, ti.haar_state(n, rng)), shots, rng)
    e, _ = L.estimate(_dev(counts), 0, flags=flags | L.LRE_NO_RHO)
    e2, _ = L.estimate(_dev(_flip_counts(n, counts, q)), 0, flags=flags | L.LRE_NO_RHO)
    e, e2 = e.cpu().numpy(), e2.cpu().numpy()
    sel = _nonidentity_at(n, q)
    assert np.max(np.abs(e2[sel] + e[sel])) <= TOL
    assert np.max(np.abs(e2[~sel] - e[~sel])) <= TOL
