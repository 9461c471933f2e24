"""Pins of the three-band part of the oracle (App. B), CPU only.

The oracle diagonalises the literal App. B matrix with numpy; these tests pin
that matrix and the table-driven Eq. (4)-(5) sum against statements that do
not go through the oracle: eigenvalues at high-symmetry momenta worked out by
hand from App. B, the filling stated in App. B, the four-state Fock-space
brute force of the pair Hamiltonian and the free-fermion normal state.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import three_band as tb
from paper_1412_8754_amd import workloads as W

M3 = W.DAGHOFER_MODEL
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def kgrid(Lx, Ly):
    kx = 2 * np.pi * np.arange(Lx) / Lx
    ky = 2 * np.pi * np.arange(Ly) / Ly
    return np.meshgrid(kx, ky, indexing="ij")


# Eigenvalues of App. B at special momenta, by hand (t1..t12, eps0 as printed):
#   Gamma (0,0): diagonal, T11 = T22 = 2t2 + 2t1 + 4t3 + 4t12 = 0.65,
#                T33 = eps0 + 4t5 + 4t6 + 4t9 + 8t10 = 1.758
#   M (pi,pi):   diagonal, T11 = T22 = -2t2 - 2t1 + 4t3 + 4t12 = 0.24,
#                T33 = eps0 - 4t5 + 4t6 + 4t9 - 8t10 = 0.942
#   X (pi,0):    diagonal, T11 = -2t2 + 2t1 - 4t3 + 4t12 = -0.75,
#                T22 = -2t1 + 2t2 - 4t3 + 4t12 = 0.30, T33 = eps0 - 4t6 + 4t9 = 0.15
#   (pi/2,pi/2): cx = cy = 0, c2x = c2y = -1: T11 = T22 = 4t12 = 0.11,
#                T33 = eps0 - 4t9 = 0.75,
#                T12 = 4t4 = -0.12, T13 = T23 = 2i t7 = -0.24i.  (1,-1,0)/sqrt2 is
#                an eigenvector with T11 - T12 = 0.23; on (1,1,0)/sqrt2, (0,0,1)
#                the matrix is [[T11 + T12, 0.24 sqrt2], [0.24 sqrt2, 0.75]] after
#                the phase change of the third orbital, with eigenvalues
#                0.37 -+ sqrt(0.38^2 + 0.1152).
SPECIAL = [
    ((0.0, 0.0), [0.65, 0.65, 1.758]),
    ((np.pi, np.pi), [0.24, 0.24, 0.942]),
    ((np.pi, 0.0), [-0.75, 0.15, 0.30]),
    ((np.pi / 2, np.pi / 2), [0.37 - math.sqrt(0.38 ** 2 + 0.1152), 0.23,
                              0.37 + math.sqrt(0.38 ** 2 + 0.1152)]),
]


@pytest.mark.parametrize("k,ref", SPECIAL)
def test_bands_at_special_momenta_worked_by_hand(k, ref):
    np.testing.assert_allclose(tb.bands(M3, *k), ref, rtol=0, atol=1e-14)


def test_filling_four_electrons_at_printed_mu():
    with open(os.path.join(GOLDEN, "three_band_filling.json")) as f:
        g = json.load(f)
    model = dict(M3, t=tuple(g["model"]["t"]), eps0=g["model"]["eps0"], mu=g["mu"])
    n = tb.filling(model, 256, 1e-4)
    assert abs(n - g["electrons_per_site"]) <= g["tolerance"], n
    # a shifted chemical potential is far from four electrons
    assert abs(tb.filling(dict(model, mu=g["mu"] + 0.05), 256, 1e-4) - 4.0) > 0.05


def test_band_symmetries():
    rng = np.random.default_rng(5)
    kx, ky = rng.uniform(-np.pi, np.pi, (2, 300))
    E = tb.bands(M3, kx, ky)
    for other in (tb.bands(M3, -kx, -ky), tb.bands(M3, ky, kx), tb.bands(M3, -kx, ky),
                  tb.bands(M3, kx + 2 * np.pi, ky)):
        np.testing.assert_allclose(other, E, rtol=0, atol=1e-13)


def fock_free_energy3(band, h, T, Lx, Ly, D, qx, qy, relative=False):
    """-T ln Tr exp(-H/T) over pair sectors (k up, -k+q down), four-state
    Fock space per sector, with App. B band energies; plus -2 Delta^2 / V.
    relative: the gap at the pair's relative momentum (k - (q - k))/2."""
    KX, KY = kgrid(Lx, Ly)
    a = tb.bands(M3, KX, KY)[..., band] - M3["mu"] - h
    b = tb.bands(M3, qx - KX, qy - KY)[..., band] - M3["mu"] + h
    if relative:
        g = D * np.cos((2 * KX - qx) / 2) * np.cos((2 * KY - qy) / 2)
    else:
        g = D * np.cos(KX) * np.cos(KY)
    H = np.zeros(KX.shape + (4, 4))
    H[..., 0, 3] = H[..., 3, 0] = g
    H[..., 1, 1] = a
    H[..., 2, 2] = b
    H[..., 3, 3] = a + b
    lam = np.linalg.eigvalsh(H)
    lo = lam.min(axis=-1)
    per_k = lo if T == 0 else lo - T * np.log(np.exp(-(lam - lo[..., None]) / T).sum(axis=-1))
    return math.fsum(per_k.ravel()) + Lx * Ly * (-2 * D * D / M3["V"][band])


@pytest.mark.parametrize("seed", range(4))
def test_three_band_free_energy_equals_fock_space_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    Lx, Ly = [(6, 8), (8, 8), (10, 6), (12, 12)][seed]
    h = rng.uniform(-0.03, 0.03)
    T = [0.0, 0.0005, 0.005, 0.05][seed]
    mq, nq = rng.integers(0, Lx), rng.integers(0, Ly)
    qx, qy = 2 * np.pi * mq / Lx, 2 * np.pi * nq / Ly
    delta = np.array([0.0, 0.01, 0.05, 0.1])
    grid = tb.omega_grid(M3, [(h, T, Lx, Ly)], delta, [[qx, qy]], tb.BAND_ALL)
    for band in range(3):
        for di, D in enumerate(delta):
            ref = fock_free_energy3(band, h, T, Lx, Ly, D, qx, qy)
            assert grid[0, band, 0, di] == pytest.approx(ref, rel=1e-12, abs=1e-13 * Lx * Ly)


@pytest.mark.parametrize("seed", range(2))
def test_three_band_relative_form_factor_equals_fock_space_brute_force(seed):
    rng = np.random.default_rng(310 + seed)
    Lx, Ly = [(8, 6), (10, 10)][seed]
    h = rng.uniform(-0.03, 0.03)
    T = [0.001, 0.02][seed]
    qx, qy = 2 * np.pi * rng.integers(1, Lx) / Lx, 2 * np.pi * rng.integers(1, Ly) / Ly
    delta = np.array([0.0, 0.03, 0.1])
    grid = tb.omega_grid(dict(M3, form=oracle.ETA_REL), [(h, T, Lx, Ly)], delta, [[qx, qy]],
                         tb.BAND_ALL)
    for band in range(3):
        for di, D in enumerate(delta):
            ref = fock_free_energy3(band, h, T, Lx, Ly, D, qx, qy, relative=True)
            assert grid[0, band, 0, di] == pytest.approx(ref, rel=1e-12, abs=1e-13 * Lx * Ly)


def test_three_band_normal_state_is_free_fermion_grand_potential():
    Lx, Ly, h, T = 10, 12, 0.02, 0.004
    E = tb.lattice_bands(M3, Lx, Ly)
    q = [[2 * np.pi * m / Lx, 2 * np.pi * n / Ly] for m, n in [(0, 0), (1, 0), (4, 7)]]
    grid = tb.omega_grid(M3, [(h, T, Lx, Ly)], [0.0], q, tb.BAND_ALL)
    for band in range(3):
        e_up = E[..., band] - M3["mu"] - h
        e_dn = E[..., band] - M3["mu"] + h
        ref = -T * (np.logaddexp(0, -e_up / T).sum() + np.logaddexp(0, -e_dn / T).sum())
        np.testing.assert_allclose(grid[0, band, :, 0], ref, rtol=1e-13)


def test_three_band_symmetries_in_q():
    # k -> -k, kx <-> ky and kx -> -kx map the App. B spectrum onto itself
    # (conjugation by diag(1,1,-1), the orbital swap 1 <-> 2, diag(-1,1,1)),
    # so Omega(q) = Omega(-q) = Omega(qy, qx) = Omega(-qx, qy) on a square
    # lattice, on or off the lattice momenta.
    L, h, T = 10, 0.02, 0.002
    rng = np.random.default_rng(8)
    delta = [0.0, 0.03, 0.08]
    for qx, qy in rng.uniform(-1, 1, size=(2, 2)):
        qs = [[qx, qy], [-qx, -qy], [qy, qx], [-qx, qy]]
        g = tb.omega_grid(M3, [(h, T, L, L)], delta, qs, tb.BAND_ALL)
        for j in range(1, 4):
            np.testing.assert_allclose(g[0, :, j, :], g[0, :, 0, :], rtol=1e-13)


def test_band_mask_selects_bands():
    pts = [(0.01, 0.001, 8, 6)]
    delta, q = [0.0, 0.04], [[0.0, 0.0], [2 * np.pi / 8, 0.0]]
    full = tb.omega_grid(M3, pts, delta, q, tb.BAND_ALL)
    for mask in (1, 2, 4, 5, 6):
        sub = tb.omega_grid(M3, pts, delta, q, mask)
        np.testing.assert_array_equal(sub, full[:, tb.band_list(mask)])


def test_row_tab_rejects_bad_inputs():
    L = oracle.lib()
    a = np.zeros(16)
    d = np.zeros(1)
    out = np.zeros(1)
    assert L.oracle_omega_row_tab(oracle._dp(a), oracle._dp(a), 4, 4, 0.0, 0.0, -1.0, -1.0,
                                  0.0, 0.0, 0, oracle._dp(d), 1, oracle._dp(out)) != 0
    assert L.oracle_omega_row_tab(oracle._dp(a), oracle._dp(a), 4, 4, 0.0, 0.0, 0.1, 0.0,
                                  0.0, 0.0, 0, oracle._dp(d), 1, oracle._dp(out)) != 0
    # no such form factor
    assert L.oracle_omega_row_tab(oracle._dp(a), oracle._dp(a), 4, 4, 0.0, 0.0, 0.1, -1.0,
                                  0.0, 0.0, 2, oracle._dp(d), 1, oracle._dp(out)) != 0
    assert L.oracle_omega_row_tab(oracle._dp(a), oracle._dp(a), 4, 4, 0.0, 0.0, 0.1, -1.0,
                                  0.0, 0.0, 1, oracle._dp(d), 1, oracle._dp(out)) == 0
