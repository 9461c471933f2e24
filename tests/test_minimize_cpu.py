"""CPU checks of the batched box-constrained quasi-Newton solver on closed-form
objectives (no GPU: the solver only needs a function returning f and g)."""
import math

import pytest

torch = pytest.importorskip("torch")

from paper_1412_8754_amd.minimize import bfgs_box  # noqa: E402


def test_many_quadratics_interior_and_on_bounds():
    # f = 0.5 (x - c)^T A (x - c) with different centres and conditioning;
    # the box clips some centres, whose solution is then the projection onto
    # the box (A diagonal here, so the projection is exact).
    P = 50
    g0 = torch.Generator().manual_seed(0)
    c = torch.rand(P, 2, generator=g0, dtype=torch.float64) * 3 - 1   # in [-1, 2]
    a = torch.rand(P, 2, generator=g0, dtype=torch.float64) * 20 + 0.1
    lo = torch.tensor([0.0, 0.0], dtype=torch.float64)
    hi = torch.tensor([1.0, 1.0], dtype=torch.float64)

    def fun(x, sel):
        r = x - c[sel]
        return 0.5 * (a[sel] * r * r).sum(dim=1), a[sel] * r

    x0 = torch.full((P, 2), 0.5, dtype=torch.float64)
    x, f, it, done = bfgs_box(fun, x0, lo, hi, max_iter=100, gtol=1e-12)
    expect = torch.minimum(torch.maximum(c, lo), hi)
    assert torch.allclose(x, expect, atol=1e-9), (x - expect).abs().max()
    assert bool(done.all())


def test_rosenbrock_valley():
    # 2-D Rosenbrock with minimum (1, 1) inside the box [-2, 2]^2
    def fun(x, sel):
        u, v = x[:, 0], x[:, 1]
        f = (1 - u) ** 2 + 100 * (v - u * u) ** 2
        g = torch.stack([-2 * (1 - u) - 400 * u * (v - u * u), 200 * (v - u * u)], dim=1)
        return f, g

    x0 = torch.tensor([[-1.2, 1.0], [0.0, 0.0], [1.8, -1.5]], dtype=torch.float64)
    lo = torch.tensor([-2.0, -2.0], dtype=torch.float64)
    hi = torch.tensor([2.0, 2.0], dtype=torch.float64)
    x, f, it, done = bfgs_box(fun, x0, lo, hi, max_iter=300, gtol=1e-10)
    assert torch.allclose(x, torch.ones_like(x), atol=1e-6), x


def test_stationary_start_on_lower_bound_is_kept():
    # f = x^2 + (y - 0.3)^2 starting at x = 0 (gradient zero in x): x stays 0
    def fun(x, sel):
        return (x[:, 0] ** 2 + (x[:, 1] - 0.3) ** 2,
                torch.stack([2 * x[:, 0], 2 * (x[:, 1] - 0.3)], dim=1))

    x0 = torch.tensor([[0.0, 0.9]], dtype=torch.float64)
    x, f, it, done = bfgs_box(fun, x0, torch.zeros(2, dtype=torch.float64),
                              torch.ones(2, dtype=torch.float64))
    assert x[0, 0] == 0.0 and abs(x[0, 1].item() - 0.3) < 1e-9


def test_function_called_only_on_unfinished_problems():
    seen = []

    def fun(x, sel):
        seen.append(sel.clone())
        return ((x - 0.25) ** 2).sum(dim=1), 2 * (x - 0.25)

    x0 = torch.tensor([[0.25, 0.25], [0.9, 0.1]], dtype=torch.float64)
    bfgs_box(fun, x0, torch.zeros(2, dtype=torch.float64), torch.ones(2, dtype=torch.float64))
    assert all(0 not in s.tolist() for s in seen[1:])


def _oracle_backend(monkeypatch):
    """Route the search's grid and gradient calls to the FP64 oracle (CPU)."""
    import numpy as np

    import oracle
    from paper_1412_8754_amd import minimize as mz

    def grid(model, pts, delta, q, bands, device=None, **kw):
        return torch.tensor(oracle.omega_grid(model, pts, delta.cpu().numpy(),
                                              q.cpu().numpy(), bands))

    def grad(model, pts, delta, q, bands, device=None, **kw):
        d = delta.cpu().numpy()
        qq = q.cpu().numpy()
        outs = [np.empty((len(pts), 2)) for _ in range(3)] + [np.empty((len(pts), 2, 2))]
        om, gd, gm, gq = outs
        for b in range(2):
            o, g1, g2, g3 = oracle.omega_grad(model, pts, d[:, b], qq[:, b], b)
            om[:, b], gd[:, b], gq[:, b], gm[:, b] = o, g1, g2, g3
        return tuple(torch.tensor(a) for a in (om, gd, gq, gm))

    monkeypatch.setattr(mz.api, "grid", grid)
    monkeypatch.setattr(mz.api, "grad", grad)
    return mz


def test_two_stage_search_reaches_lattice_grid_minimum(monkeypatch):
    import numpy as np

    import oracle
    from paper_1412_8754_amd import workloads as W
    mz = _oracle_backend(monkeypatch)
    M = W.DEFAULT_MODEL
    L = 32
    pts = W.phase_points(4, 4, fixed_L=L)
    starts, _ = mz.coarse_starts(M, pts, device="cpu")
    x, f, st = mz.minimize_points(M, pts, starts, device="cpu")
    # every lattice momentum in [0, pi/8] with a fine Delta grid (oracle)
    step = 2 * math.pi / L
    q = np.array([[m * step, 0.0] for m in range(int(math.pi / 8 / step) + 1)])
    ref = oracle.omega_grid(M, pts, np.linspace(0, 0.6, 241), q, 3)
    gmin = ref.reshape(len(pts), 2, -1).min(-1)
    f = f.numpy()
    assert (f <= gmin + 1e-12 * np.abs(gmin)).all(), (f - gmin).max()
    # the returned q are lattice momenta
    m = x[..., 1].numpy() / step
    assert np.allclose(m, np.round(m), atol=1e-9)
    assert st["converged_fraction"] == 1.0
