"""Larkin-Ovchinnikov (LO) pairing of the two-band model (test infrastructure).

Sec. 2's historical and technical note describes the LO phase as the M = 2
case of the plane-wave sum of Eq. (6): Cooper pairs of total momentum q and
-q with equal amplitude, Delta(R_j) = Delta (e^{i q.R_j} + e^{-i q.R_j}).  It
states that, with q along one lattice axis, the problem splits into
independent diagonalisations of size 2 N_y x 2 N_y, one per momentum along
the other axis.  This module writes that out plainly, with numpy's
``eigvalsh`` as the eigensolver step, for one band of App. A's model (the
bands stay independent, as in the FF case of Eq. (5)):

  Nambu modes c_{k up} and d_p = c^+_{-p down} over the zone; the 2N x 2N
  matrix has diagonal xi_up(k) = E(k) - mu - h and -xi_dn(p), xi_dn(p) =
  E(p) - mu + h (E(-p) = E(p)), and couples c_k to d_{k - q_a} with
  Delta eta(k) for each wave a (q_1 = q, q_2 = -q; one wave gives exactly
  the 2 x 2 blocks of Eq. (4) with Q = q);
  Omega_LO = -T sum_n ln(1 + e^{-E_n/T}) + sum_k xi_dn(k) - (2/V) sum_j |Delta(R_j)|^2
  over the 2N eigenvalues E_n, the second term being Eq. (5)'s sum of
  E_{k down}, the last its -2 |Delta|^2 / V per site with |Delta(R_j)|^2
  summed over the lattice sites (2 N Delta^2, or 4 N Delta^2 where 2q is a
  reciprocal lattice vector and the two waves coincide).

``omega_lo_sectors`` uses the sector decomposition the paper describes (q on
an axis); ``omega_lo_full`` diagonalises the whole 2N x 2N matrix and serves
as its brute-force check on tiny lattices.
"""
from __future__ import annotations

import math

import numpy as np


def band_energy(model, band: int, kx, ky):
    """(A.4) band energy, band 0 = E_-, 1 = E_+ (numpy, any shape)."""
    t1, t2, t3, t4 = model["t1"], model["t2"], model["t3"], model["t4"]
    cx, cy, sx, sy = np.cos(kx), np.cos(ky), np.sin(kx), np.sin(ky)
    T11 = -2.0 * (t1 * cx + t2 * cy) - 4.0 * t3 * cx * cy
    T22 = -2.0 * (t2 * cx + t1 * cy) - 4.0 * t3 * cx * cy
    T12 = -4.0 * t4 * sx * sy
    root = np.sqrt((0.5 * (T11 - T22)) ** 2 + T12 ** 2)
    return 0.5 * (T11 + T22) + (root if band else -root)


def softplus_sum(E, T: float) -> float:
    """sum_n -T ln(1 + exp(-E_n/T)) as min(E, 0) - T log1p(exp(-|E|/T));
    T = 0 gives sum min(E, 0)."""
    E = np.asarray(E, np.float64).ravel()
    lo = np.minimum(E, 0.0)
    if T == 0.0:
        return math.fsum(lo)
    return math.fsum(lo - T * np.log1p(np.exp(-np.abs(E) / T)))


def pair_weight(Lx: int, Ly: int, m: int, n: int) -> float:
    """sum_j |e^{i q.R_j} + e^{-i q.R_j}|^2 / N over the lattice sites
    R_j = (x, y), q = (2 pi m/Lx, 2 pi n/Ly): 2, or 4 where the two waves
    coincide (2q a reciprocal lattice vector)."""
    x = np.arange(Lx)[:, None]
    y = np.arange(Ly)[None, :]
    ph = 2.0 * np.pi * (m * x / Lx + n * y / Ly)
    return float(np.sum(np.abs(2.0 * np.cos(ph)) ** 2)) / (Lx * Ly)


def _constant(model, band, h, Lx, Ly, D, m, n, waves):
    """sum_k xi_dn(k) - (2/V) sum_j |Delta(R_j)|^2."""
    kx = 2.0 * np.pi * np.arange(Lx) / Lx
    ky = 2.0 * np.pi * np.arange(Ly) / Ly
    KX, KY = np.meshgrid(kx, ky, indexing="ij")
    xi_dn = band_energy(model, band, KX, KY) - model["mu"] + h
    if waves == 1:
        w = 1.0
    else:
        w = pair_weight(Lx, Ly, m, n)
    return math.fsum(xi_dn.ravel()) - 2.0 * Lx * Ly * w * D * D / model["V"][band]


def omega_lo_full(model, pt, band: int, D: float, m: int, n: int, waves: int = 2) -> float:
    """Omega_LO by diagonalising the whole 2N x 2N Nambu matrix (tiny
    lattices): q = (2 pi m/Lx, 2 pi n/Ly); waves = 1 keeps only q_1 = q (the
    FF case)."""
    h, T, Lx, Ly = pt
    N = Lx * Ly
    mu = model["mu"]
    idx = np.arange(N)
    ix, iy = idx // Ly, idx % Ly
    kx, ky = 2.0 * np.pi * ix / Lx, 2.0 * np.pi * iy / Ly
    H = np.zeros((2 * N, 2 * N))
    H[idx, idx] = band_energy(model, band, kx, ky) - mu - h
    H[N + idx, N + idx] = -(band_energy(model, band, kx, ky) - mu + h)
    eta = np.cos(kx) * np.cos(ky)
    shifts = [(m, n)] if waves == 1 else [(m, n), (-m, -n)]
    for (a, b) in shifts:
        p = ((ix - a) % Lx) * Ly + (iy - b) % Ly      # hole partner d_{k - q_a}
        H[idx, N + p] += D * eta
        H[N + p, idx] += D * eta
    E = np.linalg.eigvalsh(H)
    return softplus_sum(E, T) + _constant(model, band, h, Lx, Ly, D, m, n, waves)


def omega_lo_sectors(model, pt, band: int, delta, m: int, n: int) -> np.ndarray:
    """Omega_LO for every Delta through the paper's decomposition: with q on
    the ky axis (m = 0) one 2 Ly x 2 Ly problem per kx, with q on the kx axis
    (n = 0) one 2 Lx x 2 Lx problem per ky."""
    h, T, Lx, Ly = pt
    if m != 0 and n != 0:
        raise ValueError("q must lie on a lattice axis")
    along_y = m == 0
    Lc, Ls = (Ly, Lx) if along_y else (Lx, Ly)   # chain length, sectors
    s = n if along_y else m
    mu = model["mu"]
    kc = 2.0 * np.pi * np.arange(Lc) / Lc
    out = np.empty(len(delta))
    for di, D in enumerate(np.asarray(delta, np.float64)):
        total = 0.0
        parts = []
        for isec in range(Ls):
            ks = 2.0 * np.pi * isec / Ls
            kx, ky = (np.full(Lc, ks), kc) if along_y else (kc, np.full(Lc, ks))
            E = band_energy(model, band, kx, ky)
            H = np.zeros((2 * Lc, 2 * Lc))
            j = np.arange(Lc)
            H[j, j] = E - mu - h
            H[Lc + j, Lc + j] = -(E - mu + h)
            eta = np.cos(kx) * np.cos(ky)
            for sgn in (1, -1):
                p = (j - sgn * s) % Lc
                H[j, Lc + p] += D * eta
                H[Lc + p, j] += D * eta
            parts.append(softplus_sum(np.linalg.eigvalsh(H), T))
        total = math.fsum(parts)
        out[di] = total + _constant(model, band, h, Lx, Ly, D, m, n, 2)
    return out
