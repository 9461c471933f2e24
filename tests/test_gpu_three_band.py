"""GPU parity of the three-band model (App. B) against the FP64 oracle.

The library tabulates the eigenvalues of the App. B matrix per lattice (cyclic
Jacobi in FP64) and reads E(Q - k) from the table for lattice Q, diagonalising
at Q - k otherwise; the oracle diagonalises every momentum with numpy's
eigvalsh.  Tolerances as for the two-band model (parity_tol): FP64 1e-12
relative (plus a 1e-13 N floor), FP32-compensated 1e-7 relative, with a
2^-20 N Delta floor on lattices below 64 x 64 only (the FP32 part of each
term, P_k(Delta) - P_k(0), is at most 2 Delta); argmin indices identical.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from oracle import three_band as tb  # noqa: E402
from paper_1412_8754_amd import OMEGA_FP32_COMP, OMEGA_FP64, api  # noqa: E402
from paper_1412_8754_amd import workloads as W  # noqa: E402
from parity_tol import assert_close as _close  # noqa: E402

pytestmark = pytest.mark.gpu
M3 = W.DAGHOFER_MODEL


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def assert_close(got, ref, pts, fp32c=False, delta=None):
    return _close(got, ref, pts, fp32c=fp32c, delta=delta)


def run3(pts, delta, q, bands, prec=OMEGA_FP64):
    say(f"case: pts={pts} n_delta={len(delta)} n_q={len(q)} bands={bands} prec={prec}")
    idx, omin, rows, om = api.argmin3(M3, pts, delta, q, bands, prec)
    torch.cuda.synchronize()
    return idx.cpu().numpy(), omin.cpu().numpy(), rows.cpu().numpy(), om.cpu().numpy()


@pytest.mark.parametrize("L", [(24, 20), (64, 64), (17, 33)])
def test_band_table_matches_eigvalsh(L):
    Lx, Ly = L
    say(f"case: bands3 L={L}")
    got = api.bands3(M3, Lx, Ly).cpu().numpy()
    ref = tb.lattice_bands(M3, Lx, Ly)
    np.testing.assert_allclose(got.transpose(1, 2, 0), ref, rtol=0, atol=2e-15)


def test_three_band_grid_lattice_and_off_lattice_q():
    # Q = (2 pi/24, 0) lies on the 24 x 20 lattice but not on 16 x 16 or
    # 33 x 17; (0.1, 0.05) lies on none: both E(Q - k) paths run.  Q = 0 on
    # the square lattices (16 x 16, 37 x 37) sums the triangle j <= i of a
    # quarter of the zone.
    pts = [(0.01, 0.0005, 24, 20), (-0.02, 0.0, 16, 16), (0.005, 0.01, 33, 17),
           (0.0, 0.003, 37, 37)]
    delta = np.linspace(0.0, 0.1, 40)
    q = np.array([[0.0, 0.0], [2 * np.pi / 24, 0.0], [0.1, 0.05],
                  [2 * np.pi * 3 / 16, 2 * np.pi * 2 / 16], [2 * np.pi / 24, 2 * np.pi / 20]])
    ref = tb.omega_grid(M3, pts, delta, q, tb.BAND_ALL)
    for prec in (OMEGA_FP64, OMEGA_FP32_COMP):
        idx, omin, rows, om = run3(pts, delta, q, 7, prec)
        worst = assert_close(om, ref, pts, prec == OMEGA_FP32_COMP, delta)
        say(f"three-band grid prec={prec}: worst rel {worst:.3e}")
        if prec == OMEGA_FP64:
            ridx, romin, rrows = oracle.argmin_grid(ref)
            np.testing.assert_array_equal(idx, ridx)
            np.testing.assert_array_equal(rows, rrows)


@pytest.mark.parametrize("bands", [1, 2, 4, 5, 6])
def test_three_band_band_subsets(bands):
    pts = [(0.015, 0.002, 20, 12)]
    delta = np.linspace(0.0, 0.08, 19)
    q = np.array([[0.0, 0.0], [2 * np.pi / 20, 0.0], [0.07, 0.0]])
    ref = tb.omega_grid(M3, pts, delta, q, bands)
    om = run3(pts, delta, q, bands)[3]
    assert_close(om, ref, pts)


def test_three_band_workload_sampled_rows():
    # The three-band workload (L = 512, 128 Delta, 32 lattice Q, 3 bands) on
    # the GPU; the oracle checks 4 of the 32 Q rows of every band and the
    # argmin of each band over those rows.
    c = W.config("three_band")
    pts, delta, q = c["pts"], c["delta"], c["q"]
    idx, omin, rows, om = run3(pts, delta, q, 7)
    pick = [0, 5, 17, 31]
    ref = tb.omega_grid(M3, pts, delta, q[pick], tb.BAND_ALL)
    worst = assert_close(om[:, :, pick], ref, pts)
    say(f"three-band workload rows {pick}: worst rel {worst:.3e}")
    # the row minima agree on the sampled rows
    rr = oracle.argmin_grid(ref)[2]
    np.testing.assert_array_equal(rows[:, :, pick], rr)
    # every band has its minimum at Delta > 0 here (V puts them inside the range)
    assert (idx[0, :, 0] > 0).all()
    # the FP32-compensated grid on the same rows: 1e-7 of the oracle, same
    # row and global minima as FP64
    idx32, _, rows32, om32 = run3(pts, delta, q, 7, OMEGA_FP32_COMP)
    w32 = assert_close(om32[:, :, pick], ref, pts, True, delta)
    say(f"three-band workload fp32c rows {pick}: worst rel {w32:.3e}")
    np.testing.assert_array_equal(rows32[:, :, pick], rr)
    np.testing.assert_array_equal(idx32, idx)


def test_three_band_zone_from_symmetry_wedge():
    # Omega over every lattice pair momentum of the zone equals the wedge
    # result expanded over each orbit (GPU against GPU, and the wedge rows
    # against the oracle)
    from test_q_wedge import orbit
    Lx = Ly = 8
    pts = [(0.02, 0.002, Lx, Ly)]
    delta = np.linspace(0.0, 0.1, 12)
    qw, w = api.q_wedge(Lx, Ly)
    mn = np.rint(qw * Lx / (2 * np.pi)).astype(int)
    full_q = np.array([[2 * np.pi * m / Lx, 2 * np.pi * n / Ly]
                       for m in range(Lx) for n in range(Ly)])
    say("case: three-band wedge vs full zone 8x8")
    g_full = api.grid3(M3, pts, delta, full_q).cpu().numpy()[0]
    g_w = api.grid3(M3, pts, delta, qw).cpu().numpy()[0]
    assert_close(g_w[None], tb.omega_grid(M3, pts, delta, qw, tb.BAND_ALL), pts)
    for r, (m, n) in enumerate(mn.tolist()):
        for (a, b) in orbit(m, n, Lx, Ly):
            np.testing.assert_allclose(g_full[:, a * Ly + b], g_w[:, r], rtol=1e-12,
                                       atol=1e-13 * Lx * Ly)
