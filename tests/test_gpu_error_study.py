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
