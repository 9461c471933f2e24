"""The symmetry-reduced pair-momentum list (omega_q_wedge): host-only checks.

Each representative's orbit under the mirrors of the zone (and the diagonal
swap on square lattices) is enumerated by brute force in Python; the orbits
must partition the whole Lx x Ly lattice of pair momenta.
"""
import numpy as np
import pytest

from paper_1412_8754_amd import _abi, api


def orbit(m, n, Lx, Ly):
    pts = set()
    for sx in (1, -1):
        for sy in (1, -1):
            a, b = (sx * m) % Lx, (sy * n) % Ly
            pts.add((a, b))
            if Lx == Ly:
                pts.add((b, a))
    return pts


@pytest.mark.parametrize("Lx,Ly", [(8, 8), (7, 7), (6, 5), (2, 9), (16, 12), (64, 64)])
def test_orbits_partition_the_zone(Lx, Ly):
    q, w = api.q_wedge(Lx, Ly)
    mn = np.rint(q * np.array([Lx, Ly]) / (2 * np.pi)).astype(int)
    np.testing.assert_allclose(q, 2 * np.pi * mn / np.array([Lx, Ly]), rtol=0, atol=1e-15)
    covered = set()
    for (m, n), size in zip(mn.tolist(), w.tolist()):
        o = orbit(m, n, Lx, Ly)
        assert len(o) == size
        assert not (o & covered), "orbits overlap"
        covered |= o
    assert len(covered) == Lx * Ly
    assert int(w.sum()) == Lx * Ly
    assert mn.tolist() == sorted(mn.tolist())


def test_square_wedge_is_eighth_of_zone():
    q, w = api.q_wedge(256, 256)
    assert len(q) == 129 * 130 // 2
    assert (q[:, 1] <= q[:, 0]).all() and (q <= np.pi + 1e-15).all()


def test_wedge_errors():
    L = _abi.load()
    assert L.omega_q_wedge(1, 8, None, None, 0) == _abi.OMEGA_E_INVAL
    q = np.empty((2, 2))
    o = np.empty(2, np.int32)
    assert L.omega_q_wedge(8, 8, q.ctypes.data, o.ctypes.data, 2) == _abi.OMEGA_E_WORKSPACE
    assert L.omega_q_wedge(8, 8, q.ctypes.data, None, 2) == _abi.OMEGA_E_INVAL
