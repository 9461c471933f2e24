"""GPU: the autotuner's launch options change no result.  Calls with every
candidate option, and the tuned call, return the default call's grid and
minima bitwise (both precisions, the queued and the in-place sweeps)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1412_8754_amd import OMEGA_FP32_COMP, OMEGA_FP64, api, autotune  # noqa: E402
from paper_1412_8754_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
M = W.DEFAULT_MODEL


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def host(r):
    return [x.cpu().numpy() if x is not None else None for x in r]


def bitwise(a, b):
    for x, y in zip(a, b):
        if x is not None:
            assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


@pytest.mark.parametrize("prec", [OMEGA_FP64, OMEGA_FP32_COMP])
def test_launch_options_and_tuned_calls_are_bitwise_equal(prec, monkeypatch, tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    monkeypatch.setenv("OMEGA_TUNE_CACHE", str(tmp_path / "tune.json"))
    pts = [(0.1, 0.002, 128, 128), (0.05, 0.02, 128, 128), (0.2, 0.001, 96, 80)]
    delta = W.delta_grid(64)
    q = W.q_axis(8, 2 * np.pi / 128)
    say(f"case: launch options, prec {prec}")
    ref = host(api.argmin(M, pts, delta, q, 3, prec))
    for (b, nq) in autotune.CANDIDATES:
        got = host(api.argmin(M, pts, delta, q, 3, prec,
                              launch={"sweep_blocks_per_cu": b, "sweep_queues": nq}))
        bitwise(got, ref)
    entry = autotune.tune(M, pts, delta, q, 3, prec, reps=2)
    say(f"tuned: {entry}")
    assert autotune.lookup(pts, len(delta), len(q), 3, prec) is not None
    bitwise(host(api.argmin(M, pts, delta, q, 3, prec, tuned=True)), ref)
