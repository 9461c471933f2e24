"""C interface checks that need no GPU: the library loads, exports every
function the public header declares, and rejects invalid calls on the host
before anything is enqueued."""
import ctypes
import os
import re

import pytest

from paper_1412_8754_amd import _abi
from paper_1412_8754_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "omega.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(omega3?_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_expected_entry_points():
    assert set(header_functions()) == set(_abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _abi.load()
    for name in header_functions():
        assert hasattr(L, name), name


def test_strerror_and_version():
    assert _abi.strerror(_abi.OMEGA_OK) == "success"
    assert _abi.strerror(_abi.OMEGA_E_WORKSPACE) == "workspace too small"
    assert _abi.strerror(12345) == "unknown error code"
    assert _abi.load().omega_version() == 4


def _ws(pts, nd=8, nq=3, bands=3, prec=0, grad=0):
    return _abi.load().omega_workspace_bytes(_abi.make_points(pts), len(pts), nd, nq, bands,
                                             prec, grad)


def test_workspace_bytes_sizes():
    small = _ws([(0.0, 0.01, 16, 16)])
    big = _ws([(0.0, 0.01, 256, 256)])
    assert 0 < small < big
    # largest point dominates the per-point scratch; the grid part grows with n_pts
    two = _ws([(0.0, 0.01, 16, 16), (0.0, 0.01, 256, 256)])
    assert two > big
    assert _ws([(0.0, 0.01, 64, 64)], grad=1) > 0


@pytest.mark.parametrize("pt", [(0.0, -1e-3, 16, 16), (float("nan"), 0.01, 16, 16),
                                (0.0, float("inf"), 16, 16), (0.0, 1e-310, 16, 16),
                                (0.0, 0.01, 1, 16), (0.0, 0.01, 16, 20000),
                                (0.0, 0.01, 16384, 16384)])
def test_workspace_rejects_bad_points(pt):
    assert _ws([pt]) == 0


def test_workspace_rejects_bad_sizes():
    pts = [(0.0, 0.01, 16, 16)]
    assert _ws(pts, nd=0) == 0
    assert _ws(pts, nq=0) == 0
    assert _ws(pts, bands=0) == 0
    assert _ws(pts, bands=4) == 0
    assert _ws(pts, prec=2) == 0
    assert _abi.load().omega_workspace_bytes(None, 1, 8, 3, 3, 0, 0) == 0
    # n_q * n_delta of one (point, band) is capped at 2^30
    assert _ws(pts, nd=1 << 20, nq=1024) > 0
    assert _ws(pts, nd=1 << 20, nq=1025) == 0
    assert _ws(pts, nd=1 << 17, nq=16384) == 0


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation


def _grid(model=None, pts=None, n_pts=None, delta=FAKE, nd=8, q=FAKE, nq=3, bands=3, prec=0,
          ws=FAKE, ws_bytes=1 << 40, out=FAKE):
    L = _abi.load()
    m = _abi.make_model(model or W.DEFAULT_MODEL)
    pts = pts if pts is not None else [(0.0, 0.01, 16, 16)]
    p = _abi.make_points(pts)
    return L.omega_grid(ctypes.byref(m), p, len(pts) if n_pts is None else n_pts, delta, nd, q,
                        nq, bands, prec, ws, ws_bytes, out, None)


def test_grid_validation_errors():
    E = _abi.OMEGA_E_INVAL
    assert _grid(model=dict(W.DEFAULT_MODEL, V=(0.0, -1.0))) == E
    assert _grid(model=dict(W.DEFAULT_MODEL, mu=float("nan"))) == E
    assert _grid(pts=[(0.0, -0.1, 16, 16)]) == E
    assert _grid(n_pts=0) == E
    assert _grid(delta=None) == E
    assert _grid(q=None) == E
    assert _grid(out=None) == E
    assert _grid(ws=None) == E
    assert _grid(nd=0) == E
    assert _grid(nq=-1) == E
    assert _grid(bands=0) == E
    assert _grid(prec=7) == E
    assert _grid(ws_bytes=16) == _abi.OMEGA_E_WORKSPACE


def test_argmin_and_grad_validation_errors():
    L = _abi.load()
    m = _abi.make_model(W.DEFAULT_MODEL)
    pts = [(0.0, 0.01, 16, 16)]
    p = _abi.make_points(pts)
    big = 1 << 40
    # negative / NaN tie tolerance
    for tie in (-1.0, float("nan")):
        assert L.omega_argmin(ctypes.byref(m), p, 1, FAKE, 8, FAKE, 3, 3, 0, tie, FAKE, big,
                              FAKE, FAKE, None, None, None) == _abi.OMEGA_E_INVAL
    # missing idx output
    assert L.omega_argmin(ctypes.byref(m), p, 1, FAKE, 8, FAKE, 3, 3, 0, 1e-11, FAKE, big,
                          None, FAKE, None, None, None) == _abi.OMEGA_E_INVAL
    # no omega output: the grid needs workspace room too
    need = L.omega_workspace_bytes(p, 1, 8, 3, 3, 0, 0)
    assert L.omega_argmin(ctypes.byref(m), p, 1, FAKE, 8, FAKE, 3, 3, 0, 1e-11, FAKE, 64,
                          FAKE, FAKE, None, None, None) == _abi.OMEGA_E_WORKSPACE
    assert need > 64
    # grad: bad band mask, missing outputs, small workspace
    assert L.omega_grad(ctypes.byref(m), p, 1, FAKE, FAKE, 0, FAKE, big, FAKE, FAKE, FAKE,
                        FAKE, None) == _abi.OMEGA_E_INVAL
    assert L.omega_grad(ctypes.byref(m), p, 1, FAKE, FAKE, 3, FAKE, big, FAKE, None, FAKE,
                        FAKE, None) == _abi.OMEGA_E_INVAL
    assert L.omega_grad(ctypes.byref(m), p, 1, FAKE, FAKE, 3, FAKE, 8, FAKE, FAKE, FAKE,
                        FAKE, None) == _abi.OMEGA_E_WORKSPACE


def test_form_factor_field_is_validated():
    # a model with no such form factor is rejected before anything is enqueued
    m = _abi.make_model(dict(W.DEFAULT_MODEL, form=2))
    L = _abi.load()
    p = _abi.make_points([(0.0, 0.01, 16, 16)])
    assert L.omega_grid(ctypes.byref(m), p, 1, FAKE, 8, FAKE, 3, 3, 0, FAKE, 1 << 40, FAKE,
                        None) == _abi.OMEGA_E_INVAL
    m3 = _abi.make_model3(dict(W.DAGHOFER_MODEL, form=-1))
    assert L.omega3_grid(ctypes.byref(m3), p, 1, FAKE, 8, FAKE, 3, 7, 0, FAKE, 1 << 40, FAKE,
                         None) == _abi.OMEGA_E_INVAL


def _grid3(model=None, pts=None, delta=FAKE, nd=8, q=FAKE, nq=3, bands=7, prec=0, ws=FAKE,
           ws_bytes=1 << 40, out=FAKE):
    L = _abi.load()
    m = _abi.make_model3(model or W.DAGHOFER_MODEL)
    pts = pts if pts is not None else [(0.0, 0.001, 16, 16)]
    p = _abi.make_points(pts)
    return L.omega3_grid(ctypes.byref(m), p, len(pts), delta, nd, q, nq, bands, prec, ws,
                         ws_bytes, out, None)


def test_three_band_validation_errors():
    E = _abi.OMEGA_E_INVAL
    M3 = W.DAGHOFER_MODEL
    assert _grid3(bands=0) == E
    assert _grid3(bands=8) == E
    assert _grid3(model=dict(M3, V=(0.0, -1.0, -1.0))) == E
    # V of an unselected band is not used
    assert _grid3(model=dict(M3, V=(0.0, -1.0, -1.0)), bands=6, ws_bytes=16) == \
        _abi.OMEGA_E_WORKSPACE
    assert _grid3(model=dict(M3, eps0=float("inf"))) == E
    assert _grid3(model=dict(M3, t=(float("nan"),) + tuple(M3["t"][1:]))) == E
    assert _grid3(pts=[(0.0, 0.01, 1, 16)]) == E
    assert _grid3(out=None) == E
    assert _grid3(prec=3) == E
    assert _grid3(ws_bytes=16) == _abi.OMEGA_E_WORKSPACE
    L = _abi.load()
    m = _abi.make_model3(M3)
    p = _abi.make_points([(0.0, 0.001, 16, 16)])
    assert L.omega3_argmin(ctypes.byref(m), p, 1, FAKE, 8, FAKE, 3, 7, 0, -1.0, FAKE, 1 << 40,
                           FAKE, FAKE, None, None, None) == E
    assert L.omega3_bands(ctypes.byref(m), 1, 16, FAKE, 1 << 20, FAKE, None) == E
    assert L.omega3_bands(ctypes.byref(m), 16, 16, FAKE, 8, FAKE, None) == \
        _abi.OMEGA_E_WORKSPACE
    assert L.omega3_bands(ctypes.byref(m), 16, 16, FAKE, 1 << 20, None, None) == E


def test_three_band_workspace_holds_band_table():
    L = _abi.load()
    pts = [(0.0, 0.001, 64, 64)]
    p = _abi.make_points(pts)
    w3 = L.omega3_workspace_bytes(p, 1, 8, 3, 7, 0)
    w1 = L.omega3_workspace_bytes(p, 1, 8, 3, 1, 0)
    assert w3 > w1 > 3 * 64 * 64 * 8
    assert L.omega3_workspace_bytes(p, 1, 8, 3, 0, 0) == 0
    assert L.omega3_workspace_bytes(p, 1, 8, 3, 8, 0) == 0


def test_pair_chi_validation_errors():
    L = _abi.load()
    m = _abi.make_model(W.DEFAULT_MODEL)
    m3 = _abi.make_model3(W.DAGHOFER_MODEL)
    pts = [(0.0, 0.01, 16, 16)]
    p = _abi.make_points(pts)
    E = _abi.OMEGA_E_INVAL
    need = L.omega_chi_workspace_bytes(p, 1, 3, 3)
    assert need > 0 and L.omega3_chi_workspace_bytes(p, 1, 3, 7) > need
    assert L.omega_chi_workspace_bytes(p, 1, 0, 3) == 0
    assert L.omega_chi_workspace_bytes(p, 1, 3, 4) == 0
    assert L.omega_pair_chi(ctypes.byref(m), p, 1, FAKE, 3, 0, FAKE, 1 << 40, FAKE, None) == E
    assert L.omega_pair_chi(ctypes.byref(m), p, 1, None, 3, 3, FAKE, 1 << 40, FAKE, None) == E
    assert L.omega_pair_chi(ctypes.byref(m), p, 1, FAKE, 3, 3, FAKE, 1 << 40, None, None) == E
    assert L.omega_pair_chi(ctypes.byref(m), p, 1, FAKE, 3, 3, FAKE, 8, FAKE, None) == \
        _abi.OMEGA_E_WORKSPACE
    bad = _abi.make_points([(0.0, -1.0, 16, 16)])
    assert L.omega_pair_chi(ctypes.byref(m), bad, 1, FAKE, 3, 3, FAKE, 1 << 40, FAKE, None) == E
    # V is not used: a zero coupling is accepted (fails only on the workspace here)
    mz = _abi.make_model(dict(W.DEFAULT_MODEL, V=(0.0, 0.0)))
    assert L.omega_pair_chi(ctypes.byref(mz), p, 1, FAKE, 3, 3, FAKE, 8, FAKE, None) == \
        _abi.OMEGA_E_WORKSPACE
    assert L.omega3_pair_chi(ctypes.byref(m3), p, 1, FAKE, 3, 8, FAKE, 1 << 40, FAKE, None) == E


def test_python_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_abi, "_lib", None)
    monkeypatch.setattr(_abi, "LIB_PATH", tmp_path / "missing.so")
    with pytest.raises(RuntimeError, match="missing"):
        _abi.load()
