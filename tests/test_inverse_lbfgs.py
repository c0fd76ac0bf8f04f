"""The L-BFGS driver of the material inverse design, on CPU tensors, against
problems whose minimiser is known in closed form."""
import numpy as np
import torch

from paper_2605_14526_amd.inverse import lbfgs


def test_lbfgs_convex_quadratic_reaches_closed_form_minimiser():
    """f(x) = 1/2 x^T H x - b^T x with H SPD: the minimiser is H^-1 b."""
    rng = np.random.Generator(np.random.PCG64(7))
    n = 12
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    H = Q @ np.diag(np.logspace(0, 2, n)) @ Q.T
    b = rng.standard_normal(n)
    Ht, bt = torch.tensor(H), torch.tensor(b)

    def fg(x):
        return float(0.5 * x @ Ht @ x - bt @ x), Ht @ x - bt

    res = lbfgs(fg, torch.zeros(n, dtype=torch.float64), iters=200, memory=8, max_step=10.0, gtol=1e-12)
    xs = np.linalg.solve(H, b)
    # Armijo on f stops once decreases fall to rounding level: |x - x*| ~ sqrt(eps |f| / lambda_min)
    assert np.abs(res.x.numpy() - xs).max() < 1e-6 * np.abs(xs).max()
    assert all(a >= c for a, c in zip(res.history, res.history[1:]))  # monotone (Armijo)


def test_lbfgs_rosenbrock():
    """The Rosenbrock function's minimiser is (1, ..., 1)."""
    def fg(x):
        x = x.detach().clone().requires_grad_(True)
        f = (100.0 * (x[1:] - x[:-1] ** 2) ** 2 + (1 - x[:-1]) ** 2).sum()
        f.backward()
        return float(f), x.grad

    x0 = torch.tensor([-1.2, 1.0, -0.5, 0.8], dtype=torch.float64)
    res = lbfgs(fg, x0, iters=300, memory=6, max_step=0.5, gtol=1e-10)
    assert np.abs(res.x.numpy() - 1.0).max() < 1e-6, res.x
