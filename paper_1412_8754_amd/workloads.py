"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds input construction only (parameter grids, momentum lists,
lattice-size draws); none of the free-energy arithmetic lives here, so both the
GPU library and the CPU oracle can be fed from it without sharing any of the
method.  The workloads are parameter grids shaped like those of the paper's
Sec. 3.3 (a square N x N lattice, a Delta scan from 0 upwards, a few momenta
q along one axis, one or many (h, T) points), with the model constants of
App. A.
"""
from __future__ import annotations

import math

import numpy as np

# App. A: t1 = -1, t2 = 1.3, t3 = t4 = -0.85, mu = 1.54 (two electrons per site).
# The paper gives no V; these attractive (negative) couplings put the minima of
# both bands inside Delta in [0, 0.6] at low T.  Index 0 = E_- band, 1 = E_+.
DEFAULT_MODEL = {"t1": -1.0, "t2": 1.3, "t3": -0.85, "t4": -0.85, "mu": 1.54,
                 "V": (-16.0, -7.5)}

BAND_MINUS, BAND_PLUS, BAND_BOTH = 1, 2, 3

# App. B (three-band model of Daghofer et al.): hoppings t1..t12 and the d_xy
# on-site energy in eV as printed; mu = 0.4748 eV gives four electrons per
# site.  The paper gives no V; these put the low-T minimum of every band
# inside Delta in [0, 0.1] eV (about 0.045, 0.025 and 0.03 eV at h = 0, q = 0).
# Bands are numbered 0, 1, 2 in ascending energy; band mask bits 1, 2, 4.
DAGHOFER_MODEL = {"t": (-0.08, 0.1825, 0.08375, -0.03, 0.15, 0.15, -0.12, 0.06, 0.0,
                        -0.024, -0.01, 0.0275),
                  "eps0": 0.75, "mu": 0.4748, "V": (-4.5, -2.5, -2.0)}
BAND3_ALL = 7

# ---------------------------------------------------------------- SplitMix64
# Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
# OOPSLA 2014: state advances by the golden-ratio increment, output is the
# variant-13 finaliser.
_GAMMA = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1


def mix64(z: int) -> int:
    z &= _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def splitmix64(seed: int, counter: int) -> int:
    """The counter-th output (counter >= 1) of SplitMix64 started at seed."""
    return mix64((seed + counter * _GAMMA) & _MASK)


# ---------------------------------------------------------------- grids

def delta_grid(n: int, dmax: float = 0.6) -> np.ndarray:
    """Inclusive linspace(0, dmax, n): Algorithm 1 scans Delta from 0 to Delta_max."""
    return np.linspace(0.0, dmax, n, dtype=np.float64)


def q_axis(n: int, step: float) -> np.ndarray:
    """Q_j = (j * step, 0), j < n, as an [n][2] float64 array."""
    q = np.zeros((n, 2), np.float64)
    q[:, 0] = np.arange(n, dtype=np.float64) * step
    return q


def config(name: str) -> dict:
    """Named workloads (Delta, Q, point list, bands, precision).

    small      L=64, 128 Delta in [0,0.6], 16 q = 2 pi j / 64 along x, h=0, T=0.001
    paper      L=1024, 256 Delta, 64 q = j pi / 512 (j<64), h=0.1, T=0.002
    precision  L=2048, 512 Delta, 128 q = j pi / 1024, h=0.1, T=0.002
    three_band App. B model, L=512, 128 Delta in [0,0.1] eV, 32 q = 2 pi j / 512,
               h=0.01 eV, T=0.0005 eV, all three bands
    phase_hot  one point of the phase diagram's shape at high temperature:
               L=1024, 128 Delta, 32 q = j pi / 256, h=0.2, T=0.02
    """
    if name == "small":
        return {"name": name, "pts": [(0.0, 0.001, 64, 64)], "delta": delta_grid(128),
                "q": q_axis(16, 2.0 * math.pi / 64), "bands": BAND_BOTH}
    if name == "paper":
        return {"name": name, "pts": [(0.1, 0.002, 1024, 1024)], "delta": delta_grid(256),
                "q": q_axis(64, math.pi / 512), "bands": BAND_BOTH}
    if name == "precision":
        return {"name": name, "pts": [(0.1, 0.002, 2048, 2048)], "delta": delta_grid(512),
                "q": q_axis(128, math.pi / 1024), "bands": BAND_BOTH}
    if name == "three_band":
        return {"name": name, "pts": [(0.01, 0.0005, 512, 512)],
                "delta": delta_grid(128, 0.1), "q": q_axis(32, 2.0 * math.pi / 512),
                "bands": BAND3_ALL, "model": DAGHOFER_MODEL}
    if name == "phase_hot":
        return {"name": name, "pts": [(0.2, 0.02, 1024, 1024)], "delta": delta_grid(128),
                "q": q_axis(32, math.pi / 256), "bands": BAND_BOTH}
    raise KeyError(name)


def phase_config(n_h: int = 64, n_t: int = 64, fixed_L: int | None = None) -> dict:
    """Phase diagram: 64 x 64 (h, T) points, lattice sizes drawn per point,
    128 Delta in [0, 0.6], 32 Q = (j pi/256, 0), both bands."""
    return {"name": "phase", "pts": phase_points(n_h, n_t, fixed_L=fixed_L),
            "delta": delta_grid(128), "q": q_axis(32, math.pi / 256), "bands": BAND_BOTH}


def phase_points(n_h: int = 64, n_t: int = 64, seed: int = 0x14128754,
                 sizes=(256, 512, 1024, 2048), fixed_L: int | None = None):
    """Phase-diagram points: h in [0, 0.4], T in [1e-3, 0.05] (both linear),
    point p = n_t * a + b; L_p drawn from `sizes` by the top two bits of the
    p+1-th SplitMix64 output (or fixed_L for all points)."""
    pts = []
    for a in range(n_h):
        h = 0.4 * a / (n_h - 1) if n_h > 1 else 0.0
        for b in range(n_t):
            T = 0.001 + 0.049 * b / (n_t - 1) if n_t > 1 else 0.001
            p = n_t * a + b
            if fixed_L is None:
                L = sizes[splitmix64(seed, p + 1) >> 62]
            else:
                L = fixed_L
            pts.append((h, T, L, L))
    return pts


def random_points(rng: np.random.Generator, n: int, L_choices=(8, 12, 16),
                  h_max: float = 0.3, T_max: float = 0.05, ragged: bool = True):
    """Random (h, T, Lx, Ly) points for parity tests (Lx != Ly when ragged)."""
    pts = []
    for _ in range(n):
        Lx = int(rng.choice(L_choices))
        Ly = int(rng.choice(L_choices)) if ragged else Lx
        pts.append((float(rng.uniform(-h_max, h_max)), float(rng.uniform(0.0, T_max)),
                    Lx, Ly))
    return pts
