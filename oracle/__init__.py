"""FP64 CPU oracle for the two-band FF free energy (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  It wraps ``omega_oracle.c`` (plain C,
FP64, libm, OpenMP over the Delta loop as in the paper's CPU variant) with
ctypes and numpy.  It shares no code with the GPU library and takes no input
produced by it.

The functions follow Eq. (4)-(5) and App. A of the paper and the search of
Algorithm 1; see the header of ``omega_oracle.c`` for the readings taken where
the paper is silent.  Arrays are numpy float64 / int32, C-contiguous.
"""
from __future__ import annotations

import ctypes
import os
import pathlib
import subprocess

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_SRC = _HERE / "omega_oracle.c"
_LIB = _HERE / "liboracle.so"

BAND_MINUS = 1
BAND_PLUS = 2
BAND_BOTH = 3


class Model(ctypes.Structure):
    _fields_ = [("t1", ctypes.c_double), ("t2", ctypes.c_double),
                ("t3", ctypes.c_double), ("t4", ctypes.c_double),
                ("mu", ctypes.c_double), ("V", ctypes.c_double * 2),
                ("form", ctypes.c_int32), ("pad", ctypes.c_int32)]


# form factor of the pair (k up, -k+q down): eta(k) on the spin-up momentum
# (Sec. 2, Eq. (3)) or eta(k - q/2) at the pair's relative momentum
ETA_K, ETA_REL = 0, 1


class Point(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("T", ctypes.c_double),
                ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32)]


def build(force: bool = True) -> pathlib.Path:
    """Compile liboracle.so with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp%d" % os.getpid())
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", str(_SRC), "-o", str(tmp),
               "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _LIB.exists():
            build(force=False)
        L = ctypes.CDLL(str(_LIB))
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        mp = ctypes.POINTER(Model)
        pp = ctypes.POINTER(Point)
        L.oracle_band_energy.restype = ctypes.c_double
        L.oracle_band_energy.argtypes = [mp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.oracle_band_grad.restype = None
        L.oracle_band_grad.argtypes = [mp, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        L.oracle_omega_grid.restype = ctypes.c_int
        L.oracle_omega_grid.argtypes = [mp, pp, ctypes.c_int, dp, ctypes.c_int, dp,
                                        ctypes.c_int, ctypes.c_int, dp]
        L.oracle_argmin_grid.restype = ctypes.c_int
        L.oracle_argmin_grid.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_double, ip, dp, ip]
        L.oracle_omega_argmin.restype = ctypes.c_int
        L.oracle_omega_argmin.argtypes = [mp, pp, ctypes.c_int, dp, ctypes.c_int, dp,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ip, dp, ip, dp]
        L.oracle_omega_grad.restype = ctypes.c_int
        L.oracle_omega_grad.argtypes = [mp, pp, ctypes.c_int, dp, dp, ctypes.c_int,
                                        dp, dp, dp, dp]
        L.oracle_gap_root.restype = ctypes.c_double
        L.oracle_gap_root.argtypes = [mp, pp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_omega_row_tab.restype = ctypes.c_int
        L.oracle_omega_row_tab.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           dp, ctypes.c_int, dp]
        L.oracle_pair_chi_tab.restype = ctypes.c_int
        L.oracle_pair_chi_tab.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, dp]
        L.oracle_pair_chi.restype = ctypes.c_int
        L.oracle_pair_chi.argtypes = [mp, pp, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int, dp]
        L.oracle_max_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


# ------------------------------------------------------------------ helpers

def _model(m) -> Model:
    if isinstance(m, Model):
        return m
    return Model(m["t1"], m["t2"], m["t3"], m["t4"], m["mu"],
                 (ctypes.c_double * 2)(*m["V"]), int(m.get("form", ETA_K)), 0)


def _points(pts):
    """pts: sequence of (h, T, Lx, Ly)."""
    arr = (Point * len(pts))()
    for i, (h, T, Lx, Ly) in enumerate(pts):
        arr[i] = Point(float(h), float(T), int(Lx), int(Ly))
    return arr


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def n_bands(bands: int) -> int:
    return int(bool(bands & 1)) + int(bool(bands & 2))


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc != 0:
        raise OracleError("oracle returned %d" % rc)


# ------------------------------------------------------------------ API

def band_energy(model, band: int, kx: float, ky: float) -> float:
    """Eq. (A.4); band 0 = E_-, 1 = E_+."""
    m = _model(model)
    return lib().oracle_band_energy(ctypes.byref(m), band, kx, ky)


def band_grad(model, band: int, kx: float, ky: float):
    m = _model(model)
    gx, gy = ctypes.c_double(), ctypes.c_double()
    lib().oracle_band_grad(ctypes.byref(m), band, kx, ky, ctypes.byref(gx), ctypes.byref(gy))
    return gx.value, gy.value


def omega_grid(model, pts, delta, q, bands: int = BAND_BOTH) -> np.ndarray:
    """Omega grid [n_pts][n_bands][n_q][n_delta] (Eq. (5) per band)."""
    m = _model(model)
    p = _points(pts)
    d = _f64(delta).reshape(-1)
    qq = _f64(q).reshape(-1, 2)
    out = np.empty((len(pts), n_bands(bands), qq.shape[0], d.size), np.float64)
    _check(lib().oracle_omega_grid(ctypes.byref(m), p, len(pts), _dp(d), d.size,
                                   _dp(qq), qq.shape[0], bands, _dp(out)))
    return out


def argmin_grid(grid: np.ndarray, tie_rel: float = 1e-11):
    """Tie-ruled argmin of Algorithm 1 on a grid [..., n_q, n_delta].

    Returns (idx[..., 2] = (iDelta, iq), omin[...], row_idx[..., n_q])."""
    g = _f64(grid)
    lead = g.shape[:-2]
    n_q, n_d = g.shape[-2:]
    n_set = int(np.prod(lead)) if lead else 1
    idx = np.empty((n_set, 2), np.int32)
    omin = np.empty(n_set, np.float64)
    rows = np.empty((n_set, n_q), np.int32)
    _check(lib().oracle_argmin_grid(_dp(g), n_set, n_q, n_d, tie_rel, _ip(idx),
                                    _dp(omin), _ip(rows)))
    return idx.reshape(lead + (2,)), omin.reshape(lead), rows.reshape(lead + (n_q,))


def omega_argmin(model, pts, delta, q, bands: int = BAND_BOTH, tie_rel: float = 1e-11):
    """Grid and argmin in one call; returns (grid, idx, omin, row_idx)."""
    grid = omega_grid(model, pts, delta, q, bands)
    idx, omin, rows = argmin_grid(grid, tie_rel)
    return grid, idx, omin, rows


def omega_grad(model, pts, delta, q, band: int):
    """Per point: Omega, dOmega/dDelta, dOmega/dq[2], dOmega/dmu (band 0 or 1)."""
    m = _model(model)
    p = _points(pts)
    n = len(pts)
    d = _f64(delta).reshape(n)
    qq = _f64(q).reshape(n, 2)
    om = np.empty(n)
    gd = np.empty(n)
    gq = np.empty((n, 2))
    gm = np.empty(n)
    _check(lib().oracle_omega_grad(ctypes.byref(m), p, n, _dp(d), _dp(qq), band,
                                   _dp(om), _dp(gd), _dp(gq), _dp(gm)))
    return om, gd, gq, gm


def gap_root(model, pt, band: int, q=(0.0, 0.0), lo: float = 1e-6, hi: float = 1.0,
             tol: float = 1e-12) -> float:
    """Bisection root of dOmega/dDelta = 0 (the gap equation) on (lo, hi]."""
    m = _model(model)
    p = _points([pt])
    return lib().oracle_gap_root(ctypes.byref(m), p, band, float(q[0]), float(q[1]),
                                 lo, hi, tol)


def max_threads() -> int:
    return lib().oracle_max_threads()


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def pair_chi(model, pts, q, bands: int = BAND_BOTH) -> np.ndarray:
    """Static Cooper-pair susceptibility of App. C, two-band model:
    [n_pts][nb][nb][n_q] = chi_{eps eps'}(q) over the selected bands."""
    m = _model(model)
    p = _points(pts)
    qq = _f64(q).reshape(-1, 2)
    nb = n_bands(bands)
    out = np.empty((len(pts), nb, nb, qq.shape[0]), np.float64)
    _check(lib().oracle_pair_chi(ctypes.byref(m), p, len(pts), _dp(qq), qq.shape[0], bands,
                                 _dp(out)))
    return out
