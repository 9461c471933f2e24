"""GPU parity of the relative-momentum form factor eta(k - Q/2) (model option
OMEGA_ETA_REL) against the oracle, through the C interface: the Omega grid
and its minima for both models and precisions, on lattice and off-lattice Q,
on the mirror-folded layouts (Q on an axis, Q = 0 on a square lattice), on
both sweep kernels (below and above T = 0.005), and the gradient, whose q
derivative gains the form factor's own dependence on Q."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import three_band as tb  # noqa: E402
from paper_1412_8754_amd import OMEGA_FP32_COMP, OMEGA_FP64, api  # noqa: E402
from paper_1412_8754_amd import workloads as W  # noqa: E402
from parity_tol import assert_close, brute_argmin  # noqa: E402

pytestmark = pytest.mark.gpu
MR = dict(W.DEFAULT_MODEL, form=1)
M3R = dict(W.DAGHOFER_MODEL, form=1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("case", range(4))
def test_relative_form_factor_grid_against_oracle(case):
    Lx, Ly = [(24, 20), (33, 33), (64, 64), (17, 40)][case]
    T = [0.0, 0.002, 0.03, 0.004][case]
    pts = [(0.06, T, Lx, Ly), (-0.11, T, Lx, Ly)]
    delta = np.linspace(0.0, 0.6, [37, 16, 64, 9][case])
    q = np.array([[0.0, 0.0], [2 * np.pi * 3 / Lx, 0.0], [0.0, 2 * np.pi * 2 / Ly],
                  [2 * np.pi * 2 / Lx, 2 * np.pi * 5 / Ly], [0.27, 0.0], [0.13, -0.21]])
    ref = oracle.omega_grid(MR, pts, delta, q, 3)
    for prec in (OMEGA_FP64, OMEGA_FP32_COMP):
        say(f"case: eta(k - Q/2) {Lx}x{Ly} T={T} n_delta={len(delta)} prec={prec}")
        idx, omin, rows, om = api.argmin(MR, pts, delta, q, 3, prec)
        torch.cuda.synchronize()
        om = om.cpu().numpy()
        worst = assert_close(om, ref, pts, fp32c=prec == OMEGA_FP32_COMP, delta=delta)
        say(f"eta(k - Q/2) {Lx}x{Ly} prec {prec}: worst rel {worst:.3e}")
        idx = idx.cpu().numpy()
        for p in range(len(pts)):
            for b in range(2):
                assert tuple(idx[p, b]) == brute_argmin(ref[p, b], 1e-11), (p, b)


def test_relative_form_factor_changes_omega_off_zero_q():
    # the option is live: away from Q = 0 the two form factors give different
    # grids, at Q = 0 the same one
    pts = [(0.05, 0.003, 32, 32)]
    delta = np.linspace(0.0, 0.6, 17)
    q = np.array([[0.0, 0.0], [2 * np.pi * 4 / 32, 0.0]])
    say("case: eta(k) vs eta(k - Q/2) at L = 32")
    a = api.grid(W.DEFAULT_MODEL, pts, delta, q, 3).cpu().numpy()
    b = api.grid(MR, pts, delta, q, 3).cpu().numpy()
    np.testing.assert_array_equal(a[:, :, 0], b[:, :, 0])
    assert np.max(np.abs(a[:, :, 1, 1:] - b[:, :, 1, 1:]) / np.abs(a[:, :, 1, 1:])) > 1e-6


def test_relative_form_factor_three_band():
    pts = [(0.01, 0.0005, 24, 20), (0.0, 0.01, 16, 16)]
    delta = np.linspace(0.0, 0.1, 21)
    q = np.array([[0.0, 0.0], [2 * np.pi / 24, 0.0], [0.1, 0.05],
                  [2 * np.pi * 3 / 16, 2 * np.pi * 2 / 16]])
    ref = tb.omega_grid(M3R, pts, delta, q, tb.BAND_ALL)
    for prec in (OMEGA_FP64, OMEGA_FP32_COMP):
        say(f"case: three-band eta(k - Q/2) prec={prec}")
        idx, omin, rows, om = api.argmin3(M3R, pts, delta, q, 7, prec)
        torch.cuda.synchronize()
        worst = assert_close(om.cpu().numpy(), ref, pts, fp32c=prec == OMEGA_FP32_COMP,
                             delta=delta)
        say(f"three-band eta(k - Q/2) prec {prec}: worst rel {worst:.3e}")


@pytest.mark.parametrize("seed", range(2))
def test_relative_form_factor_gradient_against_oracle(seed):
    rng = np.random.default_rng(4000 + seed)
    n = 5
    pts = [(float(rng.uniform(-0.2, 0.2)), [0.0, 0.01, 0.05, 0.002, 0.1][i],
            int(rng.integers(4, 40)), int(rng.integers(4, 40))) for i in range(n)]
    delta = rng.uniform(0.0, 0.6, size=(n, 2))
    q = rng.uniform(-0.5, 0.5, size=(n, 2, 2))
    say(f"case: eta(k - Q/2) gradient seed {seed}")
    om, gd, gq, gm = (t.cpu().numpy() for t in api.grad(MR, pts, delta, q, 3))
    N = np.array([p[2] * p[3] for p in pts], np.float64)
    for b in range(2):
        rom, rgd, rgq, rgm = oracle.omega_grad(MR, pts, delta[:, b], q[:, b], b)
        for got, ref in ((om[:, b], rom), (gd[:, b], rgd), (gq[:, b, 0], rgq[:, 0]),
                         (gq[:, b, 1], rgq[:, 1]), (gm[:, b], rgm)):
            assert (np.abs(got - ref) <= 1e-12 * np.abs(ref) + 1e-13 * N).all(), (got, ref)


def test_relative_form_factor_paper_lattice_rows():
    # L = 1024 at the paper point: the rows Q = 0 and Q = (8 pi/512, 0) of
    # both bands against the oracle, 64 Delta, both precisions
    pts = [(0.1, 0.002, 1024, 1024)]
    delta = W.delta_grid(64)
    q = W.q_axis(16, np.pi / 512)
    import os
    oracle.set_threads(os.cpu_count() or 1)
    ref = oracle.omega_grid(MR, pts, delta, q[[0, 8]], 3)
    for prec in (OMEGA_FP64, OMEGA_FP32_COMP):
        say(f"case: eta(k - Q/2) L=1024 prec={prec}")
        om = api.grid(MR, pts, delta, q, 3, prec).cpu().numpy()
        worst = assert_close(om[:, :, [0, 8]], ref, pts, fp32c=prec == OMEGA_FP32_COMP,
                             delta=delta)
        say(f"eta(k - Q/2) L=1024 prec {prec}: worst rel {worst:.3e}")
