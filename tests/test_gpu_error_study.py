"""Estimation error of the batched estimator against its closed form (an analog of the
paper's error study, Sec. V).

For the maximally mixed state rho = I / 2^n every non-identity coefficient estimate e_i
is the average of 3^{n-w(i)} independent per-basis estimates, each of variance 1/shots
(Sec. III), and ||mu - rho||_F^2 = 2^{-n} sum_{i != 0} e_i^2 (the Omega_i are orthogonal),
so

    E ||mu - rho||_F^2 = 2^{-n} sum_{w=1}^{n} C(n, w) 3^w / (3^{n-w} shots)
                       = (10^n - 1) / (6^n shots).

M instances per (n, shots) run in one batched launch on multinomial counts drawn on the
device; the sample mean of ||mu - rho||_F^2 must match the closed form within 5 standard
errors, and each instance's value computed from mu must equal the one from its
coefficients (Parseval) to rounding.
"""
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

from paper_1602_08604_amd import lre as L  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("n,shots,m", [(3, 100, 256), (5, 300, 128), (7, 1000, 64), (9, 200, 16)])
def test_hs_error_maximally_mixed(n, shots, m):
    import tomo_inputs.gpu as tg
    print(f"[error study n={n} shots={shots} instances={m}]", flush=True)
    g = torch.Generator(device=DEV).manual_seed(1602 * 100 + n)
    p = torch.ones((3 ** n, 2 ** n), dtype=torch.float64, device=DEV)
    counts = [tg.multinomial_rows(p, shots, g) for _ in range(m)]
    b = L.Batch(counts, [shots] * m)
    b.run(check=True)
    d = 2 ** n
    eye = torch.eye(d, dtype=torch.complex128, device=DEV) / d
    hs_rho = torch.stack([((r - eye).abs() ** 2).sum() for r in b.rhos])
    hs_coef = torch.stack([(c[1:] ** 2).sum() / d for c in b.coefs])
    assert torch.max(torch.abs(hs_rho - hs_coef) / hs_coef).item() <= 1e-10
    mean = hs_rho.mean().item()
    se = hs_rho.std().item() / m ** 0.5
    expected = (10 ** n - 1) / (6 ** n * shots)
    print(f"  mean ||mu - rho||_F^2 = {mean:.6e} +- {se:.2e}; closed form {expected:.6e} "
          f"({(mean - expected) / se:+.2f} standard errors)")
    assert abs(mean - expected) <= 5 * se
    b.close()


@pytest.mark.parametrize("n,shots,m", [(4, 20, 64), (6, 50, 32)])
def test_projection_reduces_hs_error(n, shots, m):
    """Step (iii) on the same kind of instances at low shots: rho-hat is never farther
    from the true state than mu (projection onto a convex set containing it), and on
    average strictly closer (Sec. V: positivity lowers the HS error at small N_0)."""
    import tomo_inputs.gpu as tg
    print(f"[error study, step (iii), n={n} shots={shots}]", flush=True)
    g = torch.Generator(device=DEV).manual_seed(1603 * 100 + n)
    p = torch.ones((3 ** n, 2 ** n), dtype=torch.float64, device=DEV)
    counts = [tg.multinomial_rows(p, shots, g) for _ in range(m)]
    b = L.Batch(counts, [shots] * m)
    b.run(check=True)
    d = 2 ** n
    eye = torch.eye(d, dtype=torch.complex128, device=DEV) / d
    hs_mu, hs_rho = [], []
    for mu in b.rhos:
        rho, _ = L.project(mu)
        hs_mu.append(((mu - eye).abs() ** 2).sum().item())
        hs_rho.append(((rho - eye).abs() ** 2).sum().item())
    print(f"  mean HS^2: mu {sum(hs_mu) / m:.4e}, rho-hat {sum(hs_rho) / m:.4e}")
    assert all(r <= u + 1e-13 for r, u in zip(hs_rho, hs_mu))
    assert sum(hs_rho) < 0.9 * sum(hs_mu)
    b.close()


def test_infidelity_large_shots():
    """Large shots: mu is already physical, rho-hat = mu, and the infidelity to I/d,
    1 - (sum_k sqrt(lambda_k / d))^2, equals (d/4) ||rho-hat - rho||_F^2 to leading order
    (Sec. V), whose mean is (d/4) (10^n - 1)/(6^n shots) ~ (5/3)^n / (4 shots)."""
    import tomo_inputs.gpu as tg
    n, shots, m = 5, 20_000, 32
    print(f"[error study, infidelity, n={n} shots={shots}]", flush=True)
    g = torch.Generator(device=DEV).manual_seed(1604)
    p = torch.ones((3 ** n, 2 ** n), dtype=torch.float64, device=DEV)
    counts = [tg.multinomial_rows(p, shots, g) for _ in range(m)]
    b = L.Batch(counts, [shots] * m)
    b.run(check=True)
    d = 2 ** n
    eye = torch.eye(d, dtype=torch.complex128, device=DEV) / d
    infid, approx = [], []
    for mu in b.rhos:
        rho, ev = L.project(mu)
        assert ev.min().item() > 0                       # mu physical: nothing truncated
        assert torch.max(torch.abs(rho - mu)).item() <= 1e-12
        lam = torch.linalg.eigvalsh(rho).clamp_min(0)
        infid.append(1.0 - (torch.sqrt(lam / d).sum() ** 2).item())
        approx.append(d / 4 * ((rho - eye).abs() ** 2).sum().item())
    mean_inf, mean_app = sum(infid) / m, sum(approx) / m
    expected = d / 4 * (10 ** n - 1) / (6 ** n * shots)
    print(f"  mean infidelity {mean_inf:.4e}, (d/4) HS^2 {mean_app:.4e}, closed form {expected:.4e}")
    assert abs(mean_inf - mean_app) <= 0.05 * mean_app
    assert abs(mean_app - expected) <= 0.2 * expected
    b.close()
