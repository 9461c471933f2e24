"""GPU: Omega as a torch autograd function and the gradient-based search for
the minimum, against finite differences and the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1412_8754_amd import api, autodiff, minimize  # noqa: E402
from paper_1412_8754_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
M = W.DEFAULT_MODEL


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_omegafn_gradcheck_and_oracle_gradients():
    pts = [(0.05, 0.02, 12, 14), (-0.1, 0.05, 16, 10)]
    dev = "cuda"
    delta = torch.tensor([[0.2, 0.35], [0.1, 0.45]], dtype=torch.float64, device=dev,
                         requires_grad=True)
    q = torch.tensor([[[0.2, 0.0], [0.1, 0.05]], [[0.0, 0.0], [0.3, 0.0]]],
                     dtype=torch.float64, device=dev, requires_grad=True)
    mu = torch.tensor(M["mu"], dtype=torch.float64, device=dev, requires_grad=True)
    say("gradcheck of OmegaFn")
    f = lambda d, qq, m: autodiff.omega(M, pts, d, qq, m)  # noqa: E731
    assert torch.autograd.gradcheck(f, (delta, q, mu), eps=1e-6, atol=1e-5, rtol=1e-6)
    om = f(delta, q, mu)
    (om * torch.tensor([[1.0, 2.0], [3.0, 4.0]], dtype=torch.float64, device=dev)).sum().backward()
    w = np.array([[1.0, 2.0], [3.0, 4.0]])
    d_np, q_np = delta.detach().cpu().numpy(), q.detach().cpu().numpy()
    gmu = 0.0
    for b in range(2):
        rom, rgd, rgq, rgm = oracle.omega_grad(M, pts, d_np[:, b], q_np[:, b], b)
        np.testing.assert_allclose(om[:, b].detach().cpu().numpy(), rom, rtol=1e-12)
        np.testing.assert_allclose(delta.grad[:, b].cpu().numpy(), w[:, b] * rgd, rtol=1e-10, atol=1e-10)
        np.testing.assert_allclose(q.grad[:, b].cpu().numpy(), w[:, b, None] * rgq, rtol=1e-10, atol=1e-10)
        gmu += (w[:, b] * rgm).sum()
    assert mu.grad.item() == pytest.approx(gmu, rel=1e-10)


def test_torch_lbfgs_through_omegafn_finds_interior_minimum():
    # h = 0, q fixed at 0: BCS minimum in Delta (interior), via torch.optim.LBFGS
    pts = [(0.0, 0.002, 64, 64)]
    dev = "cuda"
    d = torch.tensor([[0.2, 0.2]], dtype=torch.float64, device=dev, requires_grad=True)
    q = torch.zeros((1, 2, 2), dtype=torch.float64, device=dev)
    opt = torch.optim.LBFGS([d], lr=1.0, max_iter=100, tolerance_grad=1e-12,
                            tolerance_change=1e-16, line_search_fn="strong_wolfe")

    def closure():
        opt.zero_grad()
        loss = autodiff.omega(M, pts, d, q).sum() / (64 * 64)
        loss.backward()
        return loss

    opt.step(closure)
    for b in range(2):
        root = oracle.gap_root(M, pts[0], b, (0.0, 0.0), 1e-4, 0.6)
        say(f"band {b}: LBFGS Delta {d[0, b].item():.10f}, oracle gap root {root:.10f}")
        assert abs(d[0, b].item() - root) < 1e-6


def test_batched_search_matches_oracle_grid_and_gap_equation():
    """Coarse grid -> multi-start quasi-Newton per (point, band), q snapped to
    lattice momenta, on 6 points at L = 64: the result is at least as low as
    the oracle's minimum over every lattice q in [0, pi/8] x a fine Delta grid,
    and, where Delta > 0, satisfies the gap equation."""
    pts = [(0.0, 0.001, 64, 64), (0.05, 0.002, 64, 64), (0.1, 0.002, 64, 64),
           (0.12, 0.004, 64, 64), (0.2, 0.01, 64, 64), (0.02, 0.03, 64, 64)]
    starts, _ = minimize.coarse_starts(M, pts)
    x, f, st = minimize.minimize_points(M, pts, starts)
    x, f = x.cpu().numpy(), f.cpu().numpy()
    say(f"search: {st}")
    step = 2 * math.pi / 64
    q = np.array([[m * step, 0.0] for m in range(int(math.pi / 8 / step) + 1)])
    ref = oracle.omega_grid(M, pts, np.linspace(0, 0.6, 241), q, 3)
    N = 64 * 64
    for p in range(len(pts)):
        for b in range(2):
            gmin = np.min(ref[p, b])
            om_at = oracle.omega_grid(M, [pts[p]], [x[p, b, 0]], [[x[p, b, 1], 0.0]],
                                      1 << b)[0, 0, 0, 0]
            assert om_at == pytest.approx(f[p, b], rel=1e-12)
            assert om_at <= gmin + 1e-12 * abs(gmin), (p, b, om_at, gmin)
            if x[p, b, 0] > 1e-3:
                _, gD, _, _ = oracle.omega_grad(M, [pts[p]], [x[p, b, 0]], [[x[p, b, 1], 0.0]], b)
                assert abs(gD[0]) / N < 1e-8, (p, b, gD)
