"""GPU tests of the FP64 check of the FP32-compensated search (Sec. 3.3:
scan at low precision, verify in double precision), through the C interface.

The check collects the cells whose FP32 value could lie in the FP64 tie band
of the minimum, at most 32 of them (the lowest; among equal values the
smallest keys (iDelta, iq)), re-evaluates them in FP64 and applies the tie
rule.  Grids built from repeated Delta values make many cells (nearly)
equal, which drives every branch of the selection: candidates spread over
several Q rows (groups evaluated together), Delta = 0 columns among the
cells (their values are exact FP64 ones), more than 32 equal cells under
the threshold (the scan of the whole grid in key order), and more cells
under the threshold than the LDS gather holds (2048).  The FP64 search is
checked against the oracle's grid and tie rule on the same inputs.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_1412_8754_amd import OMEGA_FP32_COMP, OMEGA_FP64, api  # noqa: E402
from paper_1412_8754_amd import workloads as W  # noqa: E402
from parity_tol import assert_close, brute_argmin  # noqa: E402

pytestmark = pytest.mark.gpu
M = W.DEFAULT_MODEL


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def both(pts, delta, q):
    out = {}
    for prec in (OMEGA_FP64, OMEGA_FP32_COMP):
        idx, omin, rows, om = api.argmin(M, pts, delta, q, 3, prec)
        torch.cuda.synchronize()
        out[prec] = (idx.cpu().numpy(), omin.cpu().numpy(), om.cpu().numpy())
    return out


# Cases whose cells under the threshold fit the 32 the check evaluates:
# the FP32-compensated search returns exactly the FP64 search's minimum.
EXACT = {
    # equal values in three Q rows (30 cells), Delta = 0 columns in the middle
    # of the grid
    "rows_and_zero_columns": ((0.02, 0.003, 40, 40),
                              np.r_[np.full(5, 0.26), [0.0], np.full(5, 0.26), [0.0, 0.1]],
                              [[0.0, 0.0], [2 * np.pi / 40, 0.0],
                               [2 * np.pi / 40, 2 * np.pi / 40]]),
    # a plain Delta scan with off-lattice and lattice Q rows
    "scan": ((0.08, 0.002, 36, 30), np.linspace(0.0, 0.6, 50),
             [[0.0, 0.0], [0.05, 0.0], [2 * np.pi / 36, 0.0], [0.0, 2 * np.pi / 30]]),
}
# Cases with more equal cells under the threshold than the check evaluates
# (exact ties at the lowest value, or more than the 2048 the gather holds):
# the FP32-compensated pick is then a cell of the FP64 tie band, with its
# FP64 Omega, though not necessarily the one of smallest key.
OVER = {
    "ties_40": ((0.05, 0.002, 48, 48), np.r_[np.zeros(1), np.full(40, 0.25), [0.4]],
                [[0.0, 0.0]]),
    "ties_2100": ((0.0, 0.004, 32, 32), np.r_[np.full(2100, 0.24), [0.0]], [[0.0, 0.0]]),
}


def check_oracle(name, pts, delta, q, out):
    i64, o64, g64 = out[OMEGA_FP64]
    _, _, g32 = out[OMEGA_FP32_COMP]
    ref = oracle.omega_grid(M, pts, delta, q, 3)
    assert_close(g64, ref, pts)
    assert_close(g32, ref, pts, fp32c=True, delta=delta)
    for b in range(2):
        assert tuple(i64[0, b]) == brute_argmin(ref[0, b], 1e-11), (name, b)


@pytest.mark.parametrize("name", sorted(EXACT))
def test_fp32c_check_returns_the_fp64_minimum(name):
    pt, delta, q = EXACT[name]
    pts = [pt]
    q = np.asarray(q, dtype=np.float64)
    say(f"case: FP64 check, {name}: L={pt[2]}x{pt[3]}, {len(delta)} Delta x {len(q)} Q")
    out = both(pts, delta, q)
    check_oracle(name, pts, delta, q, out)
    i64, o64, _ = out[OMEGA_FP64]
    i32, o32, _ = out[OMEGA_FP32_COMP]
    np.testing.assert_array_equal(i32, i64)
    np.testing.assert_allclose(o32, o64, rtol=1e-12, atol=0)
    say(f"{name}: argmin {i64.tolist()}, omin fp64 {o64.tolist()} fp32c {o32.tolist()}")


@pytest.mark.parametrize("name", sorted(OVER))
def test_fp32c_check_with_more_ties_than_it_evaluates(name):
    pt, delta, q = OVER[name]
    pts = [pt]
    q = np.asarray(q, dtype=np.float64)
    say(f"case: FP64 check, {name}: L={pt[2]}x{pt[3]}, {len(delta)} Delta x {len(q)} Q")
    out = both(pts, delta, q)
    check_oracle(name, pts, delta, q, out)
    i64, o64, g64 = out[OMEGA_FP64]
    i32, o32, _ = out[OMEGA_FP32_COMP]
    for b in range(2):
        d, iq = i32[0, b]
        assert d >= 0 and iq >= 0, (name, b)
        v64 = g64[0, b, iq, d]
        # a cell of the FP64 tie band, reported with its FP64 Omega
        assert v64 <= o64[0, b] + 1e-11 * abs(o64[0, b]), (name, b, v64, o64[0, b])
        assert abs(o32[0, b] - v64) <= 1e-12 * abs(v64), (name, b, o32[0, b], v64)
    say(f"{name}: argmin fp64 {i64.tolist()} fp32c {i32.tolist()}")
