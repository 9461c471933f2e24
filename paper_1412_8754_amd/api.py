"""Torch-facing binding of libomega: argument marshalling only.

Every function allocates its outputs (and, unless given, the workspace) as
torch CUDA tensors, passes raw device pointers and the current HIP stream to
the C interface, and returns without synchronising.  All arithmetic runs in
the library's kernels; there is no fallback path.
"""
from __future__ import annotations

import ctypes

import torch

from . import _abi
from ._abi import (OMEGA3_BAND_ALL, OMEGA_BAND_BOTH, OMEGA_FP32_COMP,  # noqa: F401
                   OMEGA_FP64, OmegaError, make_model, make_model3, make_points, n_bands,
                   n_bands3)


def _stream_ptr(stream, *tensors) -> int:
    """The HIP stream handle of a call (the current stream unless one is
    given).  On another stream, the call first waits for the work queued on
    the current stream (where its inputs were copied and its outputs and
    workspace allocated), and the call's device tensors are recorded as used
    there, so that the caching allocator does not hand their memory out again
    before that stream's work is done."""
    cur = torch.cuda.current_stream()
    s = stream if stream is not None else cur
    if s != cur:
        s.wait_stream(cur)
        for t in tensors:
            if t is not None:
                t.record_stream(s)
    return int(s.cuda_stream)


def _dev_f64(x, device, shape=None) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float64, device=device)
    if shape is not None:
        t = t.reshape(shape)
    return t.contiguous()


def _check(rc: int, what: str):
    if rc != _abi.OMEGA_OK:
        raise OmegaError(rc, what)


def workspace_bytes(pts, n_delta: int, n_q: int, bands: int = OMEGA_BAND_BOTH,
                    precision: int = OMEGA_FP64, grad: bool = False) -> int:
    L = _abi.load()
    p = make_points(pts)
    n = L.omega_workspace_bytes(p, len(pts), int(n_delta), int(n_q), int(bands),
                                int(precision), int(bool(grad)))
    if n == 0:
        raise OmegaError(_abi.OMEGA_E_INVAL, "omega_workspace_bytes")
    return int(n)


def _workspace(nbytes: int, device, workspace):
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise OmegaError(_abi.OMEGA_E_WORKSPACE, "workspace")
        return workspace
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def grid(model, pts, delta, q, bands: int = OMEGA_BAND_BOTH, precision: int = OMEGA_FP64,
         device="cuda", out=None, workspace=None, stream=None) -> torch.Tensor:
    """Omega grid [n_pts][n_bands][n_q][n_delta] (Eq. (5), Algorithm 1 loops)."""
    L = _abi.load()
    d = _dev_f64(delta, device, (-1,))
    qq = _dev_f64(q, device, (-1, 2))
    nb = n_bands(bands)
    shape = (len(pts), nb, qq.shape[0], d.numel())
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=device)
    assert out.is_contiguous() and tuple(out.shape) == shape and out.dtype == torch.float64
    ws = _workspace(workspace_bytes(pts, d.numel(), qq.shape[0], bands, precision), device,
                    workspace)
    m = make_model(model)
    p = make_points(pts)
    rc = L.omega_grid(ctypes.byref(m), p, len(pts), d.data_ptr(), d.numel(), qq.data_ptr(),
                      qq.shape[0], int(bands), int(precision), ws.data_ptr(),
                      ws.numel() * ws.element_size(), out.data_ptr(),
                      _stream_ptr(stream, d, qq, ws, out))
    _check(rc, "omega_grid")
    return out


def make_launch(launch) -> "_abi.Launch | None":
    """omega_launch from None, an _abi.Launch, or a dict with any of the keys
    sweep_blocks_per_cu, sweep_queues (launch options that change no result)."""
    if launch is None or isinstance(launch, _abi.Launch):
        return launch
    return _abi.Launch(int(launch.get("sweep_blocks_per_cu", 0)),
                       int(launch.get("sweep_queues", 0)), None, None, None)


def argmin(model, pts, delta, q, bands: int = OMEGA_BAND_BOTH, precision: int = OMEGA_FP64,
           tie_rel: float = 1e-11, keep_grid: bool = True, rows: bool = True, device="cuda",
           workspace=None, stream=None, launch=None, tuned: bool = False):
    """Grid plus the searches of Algorithm 1.

    launch: launch options (see make_launch); tuned: take them from the
    autotuner's cache for this call's shape, if it holds an entry.
    Returns (idx [n_pts][nb][2] int32 (iDelta, iq), omin [n_pts][nb],
    row_idx [n_pts][nb][n_q] or None, omega grid or None)."""
    L = _abi.load()
    if tuned and launch is None:
        from . import autotune
        launch = autotune.lookup(pts, len(delta), len(q), bands, precision)
    d = _dev_f64(delta, device, (-1,))
    qq = _dev_f64(q, device, (-1, 2))
    nb = n_bands(bands)
    n_pts, n_q, n_d = len(pts), qq.shape[0], d.numel()
    idx = torch.empty((n_pts, nb, 2), dtype=torch.int32, device=device)
    omin = torch.empty((n_pts, nb), dtype=torch.float64, device=device)
    row_idx = torch.empty((n_pts, nb, n_q), dtype=torch.int32, device=device) if rows else None
    om = torch.empty((n_pts, nb, n_q, n_d), dtype=torch.float64, device=device) if keep_grid else None
    ws = _workspace(workspace_bytes(pts, n_d, n_q, bands, precision), device, workspace)
    m = make_model(model)
    p = make_points(pts)
    lo = make_launch(launch)
    rc = L.omega_argmin_ex(ctypes.byref(m), p, n_pts, d.data_ptr(), n_d, qq.data_ptr(), n_q,
                           int(bands), int(precision), float(tie_rel), ws.data_ptr(),
                           ws.numel() * ws.element_size(), idx.data_ptr(), omin.data_ptr(),
                           row_idx.data_ptr() if row_idx is not None else None,
                           om.data_ptr() if om is not None else None,
                           ctypes.byref(lo) if lo is not None else None,
                           _stream_ptr(stream, d, qq, ws, idx, omin, row_idx, om))
    _check(rc, "omega_argmin_ex")
    return idx, omin, row_idx, om


def grad(model, pts, delta, q, bands: int = OMEGA_BAND_BOTH, device="cuda", workspace=None,
         stream=None):
    """Omega and dOmega/dDelta, dOmega/dq (2), dOmega/dmu at one (Delta, Q) per point and
    band.  delta: [n_pts][nb]; q: [n_pts][nb][2].  Returns four tensors
    ([n_pts][nb], [n_pts][nb], [n_pts][nb][2], [n_pts][nb])."""
    L = _abi.load()
    nb = n_bands(bands)
    n = len(pts)
    d = _dev_f64(delta, device, (n, nb))
    qq = _dev_f64(q, device, (n, nb, 2))
    om = torch.empty((n, nb), dtype=torch.float64, device=device)
    gd = torch.empty((n, nb), dtype=torch.float64, device=device)
    gq = torch.empty((n, nb, 2), dtype=torch.float64, device=device)
    gm = torch.empty((n, nb), dtype=torch.float64, device=device)
    ws = _workspace(workspace_bytes(pts, 1, 1, bands, OMEGA_FP64, grad=True), device, workspace)
    m = make_model(model)
    p = make_points(pts)
    rc = L.omega_grad(ctypes.byref(m), p, n, d.data_ptr(), qq.data_ptr(), int(bands),
                      ws.data_ptr(), ws.numel() * ws.element_size(), om.data_ptr(),
                      gd.data_ptr(), gq.data_ptr(), gm.data_ptr(),
                      _stream_ptr(stream, d, qq, ws, om, gd, gq, gm))
    _check(rc, "omega_grad")
    return om, gd, gq, gm


# ------------------------------------------------------------- LO pairing

def lo_grid(model, pts, delta, q_index, bands: int = OMEGA_BAND_BOTH, device="cuda",
            workspace=None, stream=None) -> torch.Tensor:
    """Omega of the LO state (pair momenta q and -q, equal amplitude) of the
    two-band model, [n_pts][nb][n_q][n_delta]; q_index: [n_q][2] lattice
    indices (m, n) of q = (2 pi m/Lx, 2 pi n/Ly), one of them 0."""
    import numpy as np
    L = _abi.load()
    d = _dev_f64(delta, device, (-1,))
    qi = np.ascontiguousarray(np.asarray(q_index, dtype=np.int32).reshape(-1, 2))
    nb = n_bands(bands)
    p = make_points(pts)
    n = L.omega_lo_workspace_bytes(p, len(pts), d.numel(), qi.ctypes.data, qi.shape[0],
                                   int(bands))
    if n == 0:
        raise OmegaError(_abi.OMEGA_E_UNSUPPORTED, "omega_lo_workspace_bytes")
    ws = _workspace(int(n), device, workspace)
    out = torch.empty((len(pts), nb, qi.shape[0], d.numel()), dtype=torch.float64,
                      device=device)
    m = make_model(model)
    rc = L.omega_lo_grid(ctypes.byref(m), p, len(pts), d.data_ptr(), d.numel(),
                         qi.ctypes.data, qi.shape[0], int(bands), ws.data_ptr(),
                         ws.numel() * ws.element_size(), out.data_ptr(),
                         _stream_ptr(stream, d, ws, out))
    _check(rc, "omega_lo_grid")
    return out


# ------------------------------------------------------------- three-band model

def bands3(model, Lx: int, Ly: int, device="cuda", stream=None) -> torch.Tensor:
    """Band table of App. B on the Lx x Ly lattice, [3][Lx][Ly], ascending."""
    L = _abi.load()
    out = torch.empty((3, int(Lx), int(Ly)), dtype=torch.float64, device=device)
    ws = torch.empty(16 * (int(Lx) + int(Ly)), dtype=torch.uint8, device=device)
    m = make_model3(model)
    rc = L.omega3_bands(ctypes.byref(m), int(Lx), int(Ly), ws.data_ptr(), ws.numel(),
                        out.data_ptr(), _stream_ptr(stream, ws, out))
    _check(rc, "omega3_bands")
    return out


def workspace_bytes3(pts, n_delta: int, n_q: int, bands: int = OMEGA3_BAND_ALL,
                     precision: int = OMEGA_FP64) -> int:
    L = _abi.load()
    p = make_points(pts)
    n = L.omega3_workspace_bytes(p, len(pts), int(n_delta), int(n_q), int(bands),
                                 int(precision))
    if n == 0:
        raise OmegaError(_abi.OMEGA_E_INVAL, "omega3_workspace_bytes")
    return int(n)


def grid3(model, pts, delta, q, bands: int = OMEGA3_BAND_ALL, precision: int = OMEGA_FP64,
          device="cuda", out=None, workspace=None, stream=None) -> torch.Tensor:
    """Three-band Omega grid [n_pts][n_bands][n_q][n_delta]."""
    L = _abi.load()
    d = _dev_f64(delta, device, (-1,))
    qq = _dev_f64(q, device, (-1, 2))
    nb = n_bands3(bands)
    shape = (len(pts), nb, qq.shape[0], d.numel())
    if out is None:
        out = torch.empty(shape, dtype=torch.float64, device=device)
    assert out.is_contiguous() and tuple(out.shape) == shape and out.dtype == torch.float64
    ws = _workspace(workspace_bytes3(pts, d.numel(), qq.shape[0], bands, precision), device,
                    workspace)
    m = make_model3(model)
    p = make_points(pts)
    rc = L.omega3_grid(ctypes.byref(m), p, len(pts), d.data_ptr(), d.numel(), qq.data_ptr(),
                       qq.shape[0], int(bands), int(precision), ws.data_ptr(),
                       ws.numel() * ws.element_size(), out.data_ptr(),
                       _stream_ptr(stream, d, qq, ws, out))
    _check(rc, "omega3_grid")
    return out


def argmin3(model, pts, delta, q, bands: int = OMEGA3_BAND_ALL, precision: int = OMEGA_FP64,
            tie_rel: float = 1e-11, keep_grid: bool = True, rows: bool = True,
            device="cuda", workspace=None, stream=None):
    """Three-band grid plus the searches of Algorithm 1 (outputs as argmin)."""
    L = _abi.load()
    d = _dev_f64(delta, device, (-1,))
    qq = _dev_f64(q, device, (-1, 2))
    nb = n_bands3(bands)
    n_pts, n_q, n_d = len(pts), qq.shape[0], d.numel()
    idx = torch.empty((n_pts, nb, 2), dtype=torch.int32, device=device)
    omin = torch.empty((n_pts, nb), dtype=torch.float64, device=device)
    row_idx = torch.empty((n_pts, nb, n_q), dtype=torch.int32, device=device) if rows else None
    om = torch.empty((n_pts, nb, n_q, n_d), dtype=torch.float64, device=device) if keep_grid else None
    ws = _workspace(workspace_bytes3(pts, n_d, n_q, bands, precision), device, workspace)
    m = make_model3(model)
    p = make_points(pts)
    rc = L.omega3_argmin(ctypes.byref(m), p, n_pts, d.data_ptr(), n_d, qq.data_ptr(), n_q,
                         int(bands), int(precision), float(tie_rel), ws.data_ptr(),
                         ws.numel() * ws.element_size(), idx.data_ptr(), omin.data_ptr(),
                         row_idx.data_ptr() if row_idx is not None else None,
                         om.data_ptr() if om is not None else None,
                         _stream_ptr(stream, d, qq, ws, idx, omin, row_idx, om))
    _check(rc, "omega3_argmin")
    return idx, omin, row_idx, om


# ------------------------------------------------------------- Q wedge

def q_wedge(Lx: int, Ly: int):
    """Lattice pair momenta of the whole zone reduced by symmetry (host only):
    returns (q [n][2] float64 numpy, orbit [n] int32 numpy); the orbit sizes
    add up to Lx * Ly."""
    import numpy as np
    L = _abi.load()
    n = L.omega_q_wedge(int(Lx), int(Ly), None, None, 0)
    _check(min(n, 0), "omega_q_wedge")
    q = np.empty((n, 2), np.float64)
    orbit = np.empty(n, np.int32)
    rc = L.omega_q_wedge(int(Lx), int(Ly), q.ctypes.data, orbit.ctypes.data, n)
    _check(min(rc, 0), "omega_q_wedge")
    return q, orbit


# ------------------------------------------------------------- App. C

def pair_chi(model, pts, q, bands: int = OMEGA_BAND_BOTH, device="cuda", workspace=None,
             stream=None) -> torch.Tensor:
    """Static Cooper-pair susceptibility of App. C, two-band model:
    [n_pts][nb][nb][n_q] = chi_{eps eps'}(q)."""
    L = _abi.load()
    qq = _dev_f64(q, device, (-1, 2))
    nb = n_bands(bands)
    p = make_points(pts)
    n = L.omega_chi_workspace_bytes(p, len(pts), qq.shape[0], int(bands))
    if n == 0:
        raise OmegaError(_abi.OMEGA_E_INVAL, "omega_chi_workspace_bytes")
    ws = _workspace(int(n), device, workspace)
    out = torch.empty((len(pts), nb, nb, qq.shape[0]), dtype=torch.float64, device=device)
    m = make_model(model)
    rc = L.omega_pair_chi(ctypes.byref(m), p, len(pts), qq.data_ptr(), qq.shape[0], int(bands),
                          ws.data_ptr(), ws.numel() * ws.element_size(), out.data_ptr(),
                          _stream_ptr(stream, qq, ws, out))
    _check(rc, "omega_pair_chi")
    return out


def pair_chi3(model, pts, q, bands: int = OMEGA3_BAND_ALL, device="cuda", workspace=None,
              stream=None) -> torch.Tensor:
    """Static Cooper-pair susceptibility of App. C, three-band model."""
    L = _abi.load()
    qq = _dev_f64(q, device, (-1, 2))
    nb = n_bands3(bands)
    p = make_points(pts)
    n = L.omega3_chi_workspace_bytes(p, len(pts), qq.shape[0], int(bands))
    if n == 0:
        raise OmegaError(_abi.OMEGA_E_INVAL, "omega3_chi_workspace_bytes")
    ws = _workspace(int(n), device, workspace)
    out = torch.empty((len(pts), nb, nb, qq.shape[0]), dtype=torch.float64, device=device)
    m = make_model3(model)
    rc = L.omega3_pair_chi(ctypes.byref(m), p, len(pts), qq.data_ptr(), qq.shape[0],
                           int(bands), ws.data_ptr(), ws.numel() * ws.element_size(),
                           out.data_ptr(), _stream_ptr(stream, qq, ws, out))
    _check(rc, "omega3_pair_chi")
    return out
