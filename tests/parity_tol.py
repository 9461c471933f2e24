"""Parity tolerances of the GPU path against the FP64 oracle (test-side).

FP64 path: |dOmega| <= 1e-12 |Omega| + 1e-13 N elementwise (N = Lx*Ly; the
floor only matters where Omega passes through zero).

FP32-compensated path: |dOmega| <= 1e-7 |Omega| against the oracle, the error
the precision pattern promises, on every lattice of at least 64 x 64
momenta, with one qualification: Omega of the E_+ band rises through zero at
large Delta (the -2 Delta^2 N / V term overtakes the rest), where no relative
bound can hold, so |Omega| is taken as at least the largest |Omega| of the
compared cells of its Q row (the scale of the terms being summed; for the
E_- band, and for E_+ away from the crossing, that is |Omega| itself).  Only
on smaller lattices, where the sum over k can cancel to an Omega far
smaller than its terms, is a floor added: 2^-20 N |Delta|.  It
follows from the precision split: only P_k(Delta) - P_k(0) is computed in
FP32, and it is at most 2 Delta per momentum (each branch energy of Eq. (4)
moves by at most Delta |eta| <= Delta, and T ln(1 + e^-E/T) is 1-Lipschitz
in E), so a few FP32 ulps of it (2^-24 x 8 x 2 Delta) bound the error per
site.  A 3 x 3 lattice at Delta = 0.6, whose Omega cancels to 0.28, needs it.
"""
import numpy as np

FP32C_NO_FLOOR_SITES = 64 * 64


def n_sites(pts):
    return np.array([p[2] * p[3] for p in pts], dtype=np.float64)


def assert_close(got, ref, pts, fp32c=False, delta=None, rel=None):
    """Elementwise check of got against the oracle's ref, with the points on
    the first axis and Delta on the last; returns the worst relative error
    (FP32-compensated: relative to the scale above)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    N = n_sites(pts).reshape((-1,) + (1,) * (ref.ndim - 1))
    err = np.abs(got - ref)
    if not fp32c:
        tol = (1e-12 if rel is None else rel) * np.abs(ref) + 1e-13 * N
    else:
        scale = np.maximum(np.abs(ref), np.max(np.abs(ref), axis=-1, keepdims=True))
        tol = (1e-7 if rel is None else rel) * scale
        small = N < FP32C_NO_FLOOR_SITES
        if small.any():
            assert delta is not None, "the small-lattice floor needs the Delta values"
            d = np.abs(np.asarray(delta, dtype=np.float64))
            tol = tol + np.where(small, 2.0 ** -20 * N * d, 0.0)
    bad = err > tol
    den = np.abs(ref) if not fp32c else scale
    worst = float(np.max(err / (den + 1e-300))) if err.size else 0.0
    assert not bad.any(), f"{int(bad.sum())} mismatches, worst rel {worst:.3e}"
    return worst


def brute_argmin(g, tie):
    """Tie rule of Algorithm 1's search, written out in plain Python over a
    [n_q][n_delta] grid: among the non-NaN points with Omega <= min + tie |min|
    the lexicographically smallest (iDelta, iq)."""
    ok = ~np.isnan(g)
    if not ok.any():
        return (-1, -1)
    best = np.min(g[ok])
    thr = best + tie * abs(best)
    cand = [(idl, iq) for iq in range(g.shape[0]) for idl in range(g.shape[1])
            if ok[iq, idl] and g[iq, idl] <= thr]
    return min(cand)
