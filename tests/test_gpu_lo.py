"""GPU parity of the LO pairing (two plane waves q and -q) against the
oracle's sector decomposition, through the C interface: lattice q on either
axis, cycles of 2 to 128 modes (the three kernel sizes), q = 0 and 2q = 0
(where the two waves coincide), T = 0 and finite T, both bands; FP64 within
1e-12 of the oracle."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import lo_phase as lo  # noqa: E402
from paper_1412_8754_amd import api  # noqa: E402
from paper_1412_8754_amd import workloads as W  # noqa: E402
from parity_tol import assert_close  # noqa: E402

pytestmark = pytest.mark.gpu
M = W.DEFAULT_MODEL


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("case", range(5))
def test_lo_grid_against_oracle(case):
    pts, qi = [
        ([(0.05, 0.01, 16, 16), (-0.1, 0.0, 16, 16)], [[0, 0], [1, 0], [0, 3], [8, 0], [0, 4]]),
        ([(0.12, 0.002, 24, 20)], [[1, 0], [0, 1], [6, 0], [0, 5]]),
        ([(0.0, 0.03, 128, 6)], [[1, 0], [3, 0], [0, 2]]),        # 128-mode cycles
        ([(0.07, 0.005, 9, 33)], [[0, 1], [2, 0], [0, 11]]),      # odd sides: 66-mode cycles
        ([(0.2, 0.0, 32, 32)], [[2, 0], [0, 16], [5, 0]]),
    ][case]
    delta = np.linspace(0.0, 0.6, [9, 7, 5, 6, 8][case])
    say(f"case: LO pts={pts} q={qi} n_delta={len(delta)}")
    got = api.lo_grid(M, pts, delta, qi, 3).cpu().numpy()
    ref = np.empty_like(got)
    for p, pt in enumerate(pts):
        for b in range(2):
            for iq, (m, n) in enumerate(qi):
                ref[p, b, iq] = lo.omega_lo_sectors(M, pt, b, delta, m, n)
    worst = assert_close(got, ref, pts)
    say(f"LO case {case}: worst rel {worst:.3e}")


def test_lo_single_band_and_rejections():
    pts = [(0.05, 0.01, 16, 16)]
    delta = np.array([0.0, 0.3])
    say("case: LO band subsets and rejected requests")
    both = api.lo_grid(M, pts, delta, [[2, 0]], 3).cpu().numpy()
    for bands, sl in ((1, 0), (2, 1)):
        one = api.lo_grid(M, pts, delta, [[2, 0]], bands).cpu().numpy()
        assert np.array_equal(one[:, 0], both[:, sl])
    from paper_1412_8754_amd import OmegaError
    with pytest.raises(OmegaError):
        api.lo_grid(M, pts, delta, [[1, 1]], 3)          # q off the axes
    with pytest.raises(OmegaError):
        api.lo_grid(M, [(0.0, 0.01, 200, 8)], delta, [[1, 0]], 3)   # a 400-mode cycle
