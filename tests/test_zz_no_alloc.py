"""omega_argmin_noalloc (scratch in the library's static device array)
against omega_argmin (caller's workspace), through the C interface.

Two calls in a row on the same device, the second with a smaller input, so
the second reads an array the first has left filled; each must give the
workspace call's results bitwise (the same kernels run on the same inputs).
Also: a request beyond the array's size is refused with OMEGA_E_WORKSPACE
before anything is enqueued, and invalid arguments with OMEGA_E_INVAL.
"""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1412_8754_amd import _abi  # noqa: E402
from paper_1412_8754_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _call(fn_name, pts, delta, q, bands, precision, keep_grid):
    L = _abi.load()
    dev = torch.device("cuda:0")
    d = torch.as_tensor(delta, dtype=torch.float64, device=dev).contiguous()
    qq = torch.as_tensor(q, dtype=torch.float64, device=dev).reshape(-1, 2).contiguous()
    nb = _abi.n_bands(bands)
    n_pts, n_q, n_d = len(pts), qq.shape[0], d.numel()
    idx = torch.full((n_pts, nb, 2), -7, dtype=torch.int32, device=dev)
    omin = torch.full((n_pts, nb), float("nan"), dtype=torch.float64, device=dev)
    rows = torch.full((n_pts, nb, n_q), -7, dtype=torch.int32, device=dev)
    om = (torch.full((n_pts, nb, n_q, n_d), float("nan"), dtype=torch.float64, device=dev)
          if keep_grid else None)
    m = _abi.make_model(W.DEFAULT_MODEL)
    p = _abi.make_points(pts)
    s = torch.cuda.current_stream().cuda_stream
    if fn_name == "omega_argmin":
        nbytes = L.omega_workspace_bytes(p, n_pts, n_d, n_q, bands, precision, 0)
        assert nbytes > 0
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        rc = L.omega_argmin(ctypes.byref(m), p, n_pts, d.data_ptr(), n_d, qq.data_ptr(), n_q,
                            bands, precision, 1e-11, ws.data_ptr(), nbytes, idx.data_ptr(),
                            omin.data_ptr(), rows.data_ptr(),
                            om.data_ptr() if om is not None else None, s)
    else:
        rc = L.omega_argmin_noalloc(ctypes.byref(m), p, n_pts, d.data_ptr(), n_d,
                                    qq.data_ptr(), n_q, bands, precision, 1e-11,
                                    idx.data_ptr(), omin.data_ptr(), rows.data_ptr(),
                                    om.data_ptr() if om is not None else None, s)
    assert rc == _abi.OMEGA_OK, (fn_name, rc, _abi.strerror(rc))
    torch.cuda.synchronize()
    out = [idx.cpu().numpy(), omin.cpu().numpy(), rows.cpu().numpy()]
    if om is not None:
        out.append(om.cpu().numpy())
    return out


CASES = [
    # larger first, then smaller: the second call finds the first's data in
    # the shared array
    ("two points, 48 Delta x 6 Q", [(0.1, 0.002, 64, 48), (0.02, 0.03, 40, 40)],
     W.delta_grid(48), W.q_axis(6, 2 * np.pi / 40), 3),
    ("one point, 20 Delta x 3 Q", [(0.05, 0.004, 24, 20)], W.delta_grid(20),
     W.q_axis(3, 2 * np.pi / 24), 3),
]


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("keep_grid", [True, False])
def test_noalloc_matches_workspace_call_on_consecutive_calls(precision, keep_grid):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    for name, pts, delta, q, bands in CASES:
        say(f"case: {name}, precision {precision}, keep_grid {keep_grid}")
        got = _call("omega_argmin_noalloc", pts, delta, q, bands, precision, keep_grid)
        ref = _call("omega_argmin", pts, delta, q, bands, precision, keep_grid)
        for g, r in zip(got, ref):
            np.testing.assert_array_equal(g, r)


def test_noalloc_refuses_what_does_not_fit_and_invalid_arguments():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    L = _abi.load()
    m = _abi.make_model(W.DEFAULT_MODEL)
    pts = [(0.1, 0.002, 4096, 4096)]
    p = _abi.make_points(pts)
    need = L.omega_workspace_bytes(p, 1, 256, 64, 3, 0, 0)
    assert need > _abi.OMEGA_NOALLOC_SCRATCH_BYTES
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: refused before any launch
    rc = L.omega_argmin_noalloc(ctypes.byref(m), p, 1, fake, 256, fake, 64, 3, 0, 1e-11,
                                fake, fake, None, fake, None)
    assert rc == _abi.OMEGA_E_WORKSPACE
    rc = L.omega_argmin_noalloc(ctypes.byref(m), p, 1, fake, 256, fake, 64, 4, 0, 1e-11,
                                fake, fake, None, fake, None)
    assert rc == _abi.OMEGA_E_INVAL
    small = _abi.make_points([(0.1, 0.002, 16, 16)])
    rc = L.omega_argmin_noalloc(ctypes.byref(m), small, 1, fake, 8, fake, 2, 3, 0, -1.0,
                                fake, fake, None, fake, None)
    assert rc == _abi.OMEGA_E_INVAL
