"""Three-band (Daghofer et al.) part of the oracle: App. B (test infrastructure).

The band energies are the eigenvalues of the 3x3 orbital hopping matrix of
App. B, written out literally as a complex Hermitian matrix and diagonalised
with numpy's ``eigvalsh`` (a library routine, used as one step).  Bands are
numbered 0, 1, 2 in ascending order of energy at each k.  The free energy of
each band then follows Eq. (4)-(5) exactly as for the two-band model, through
the table-driven C routine ``oracle_omega_row_tab``; E_eps(q - k) is
diagonalised at q - k itself (no lattice shift).

Model: dict with "t" (t1..t12, eV), "eps0" (on-site energy of d_xy), "mu",
"V" (three couplings, one per band; V < 0 attractive), and optionally "form"
(the form factor: 0 = eta(k), 1 = eta(k - q/2); see the two-band oracle).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _check, _dp, _f64, lib

BAND_0, BAND_1, BAND_2 = 1, 2, 4
BAND_ALL = 7


def band_list(bands: int):
    return [b for b in range(3) if bands & (1 << b)]


def hamiltonian(model, kx, ky) -> np.ndarray:
    """App. B orbital matrix T_k (d_xz, d_yz, d_xy), shape [..., 3, 3]."""
    t = [None] + list(model["t"])        # t[1] .. t[12]
    e0 = model["eps0"]
    kx = np.asarray(kx, np.float64)
    ky = np.asarray(ky, np.float64)
    cx, cy, sx, sy = np.cos(kx), np.cos(ky), np.sin(kx), np.sin(ky)
    c2x, c2y = np.cos(2 * kx), np.cos(2 * ky)
    H = np.zeros(np.broadcast(kx, ky).shape + (3, 3), np.complex128)
    H[..., 0, 0] = (2 * t[2] * cx + 2 * t[1] * cy + 4 * t[3] * cx * cy
                    + 2 * t[11] * (c2x - c2y) + 4 * t[12] * c2x * c2y)
    H[..., 1, 1] = (2 * t[1] * cx + 2 * t[2] * cy + 4 * t[3] * cx * cy
                    - 2 * t[11] * (c2x - c2y) + 4 * t[12] * c2x * c2y)
    H[..., 2, 2] = (e0 + 2 * t[5] * (cx + cy) + 4 * t[6] * cx * cy
                    + 2 * t[9] * (c2x + c2y) + 4 * t[10] * (c2x * cy + cx * c2y))
    H[..., 0, 1] = H[..., 1, 0] = 4 * t[4] * sx * sy
    H[..., 0, 2] = 2j * t[7] * sx + 4j * t[8] * sx * cy
    H[..., 2, 0] = np.conj(H[..., 0, 2])
    H[..., 1, 2] = 2j * t[7] * sy + 4j * t[8] * sy * cx
    H[..., 2, 1] = np.conj(H[..., 1, 2])
    return H


def bands(model, kx, ky) -> np.ndarray:
    """Band energies E_0 <= E_1 <= E_2 at (kx, ky), shape [..., 3]."""
    return np.linalg.eigvalsh(hamiltonian(model, kx, ky))


def lattice_bands(model, Lx: int, Ly: int) -> np.ndarray:
    """E_eps(k) on the lattice kx = 2 pi i/Lx, ky = 2 pi j/Ly, [Lx, Ly, 3]."""
    kx = 2 * np.pi * np.arange(Lx) / Lx
    ky = 2 * np.pi * np.arange(Ly) / Ly
    KX, KY = np.meshgrid(kx, ky, indexing="ij")
    return bands(model, KX, KY)


def filling(model, L: int, T: float, h: float = 0.0) -> float:
    """Electrons per site, sum over the three bands and both spins of the Fermi
    function of E_eps(k) - mu -+ h, on an L x L lattice."""
    E = lattice_bands(model, L, L)
    n = 0.0
    for sgn in (1.0, -1.0):
        x = (E - model["mu"] - sgn * h) / T
        n += np.sum(0.5 * (1.0 - np.tanh(0.5 * x)))
    return n / (L * L)


def omega_grid(model, pts, delta, q, bands_mask: int = BAND_ALL) -> np.ndarray:
    """Omega grid [n_pts][n_bands][n_q][n_delta] of the three-band model
    (Eq. (5) per band, energies from App. B)."""
    d = _f64(delta).reshape(-1)
    qq = _f64(q).reshape(-1, 2)
    bl = band_list(bands_mask)
    out = np.empty((len(pts), len(bl), qq.shape[0], d.size), np.float64)
    L = lib()
    for p, (h, T, Lx, Ly) in enumerate(pts):
        kx = 2 * np.pi * np.arange(Lx) / Lx
        ky = 2 * np.pi * np.arange(Ly) / Ly
        KX, KY = np.meshgrid(kx, ky, indexing="ij")
        ek = bands(model, KX, KY)
        for iq in range(qq.shape[0]):
            eqk = bands(model, qq[iq, 0] - KX, qq[iq, 1] - KY)
            for ib, b in enumerate(bl):
                a = np.ascontiguousarray(ek[..., b])
                c = np.ascontiguousarray(eqk[..., b])
                row = np.empty(d.size, np.float64)
                _check(L.oracle_omega_row_tab(_dp(a), _dp(c), int(Lx), int(Ly),
                                              float(model["mu"]), float(h), float(T),
                                              float(model["V"][b]), float(qq[iq, 0]),
                                              float(qq[iq, 1]), int(model.get("form", 0)),
                                              _dp(d), d.size, _dp(row)))
                out[p, ib, iq] = row
    return out


def pair_chi(model, pts, q, bands_mask: int = BAND_ALL) -> np.ndarray:
    """Static Cooper-pair susceptibility of App. C for the three-band model:
    [n_pts][nb][nb][n_q] = chi_{eps eps'}(q), E_eps'(-k-q) diagonalised at
    -k-q."""
    qq = _f64(q).reshape(-1, 2)
    bl = band_list(bands_mask)
    out = np.empty((len(pts), len(bl), len(bl), qq.shape[0]), np.float64)
    L = lib()
    for p, (h, T, Lx, Ly) in enumerate(pts):
        kx = 2 * np.pi * np.arange(Lx) / Lx
        ky = 2 * np.pi * np.arange(Ly) / Ly
        KX, KY = np.meshgrid(kx, ky, indexing="ij")
        ek = bands(model, KX, KY)
        for iq in range(qq.shape[0]):
            e2 = bands(model, -KX - qq[iq, 0], -KY - qq[iq, 1])
            for ia, a in enumerate(bl):
                for ib, b in enumerate(bl):
                    x = np.ascontiguousarray(ek[..., a])
                    y = np.ascontiguousarray(e2[..., b])
                    r = np.empty(1, np.float64)
                    _check(L.oracle_pair_chi_tab(_dp(x), _dp(y), int(Lx), int(Ly),
                                                 float(model["mu"]), float(h), float(T),
                                                 float(qq[iq, 0]), float(qq[iq, 1]), _dp(r)))
                    out[p, ia, ib, iq] = r[0]
    return out
