"""ctypes view of libomega's C interface (include/omega.h); no torch here."""
from __future__ import annotations

import ctypes
import pathlib

PKG = pathlib.Path(__file__).resolve().parent
LIB_PATH = PKG / "libomega.so"

OMEGA_BAND_MINUS, OMEGA_BAND_PLUS, OMEGA_BAND_BOTH = 1, 2, 3
OMEGA_FP64, OMEGA_FP32_COMP = 0, 1
OMEGA_OK, OMEGA_E_INVAL, OMEGA_E_WORKSPACE, OMEGA_E_HIP, OMEGA_E_UNSUPPORTED = 0, -1, -2, -3, -4

OMEGA3_BAND_0, OMEGA3_BAND_1, OMEGA3_BAND_2, OMEGA3_BAND_ALL = 1, 2, 4, 7
OMEGA_NOALLOC_SCRATCH_BYTES = 128 << 20

EXPORTS = ("omega_workspace_bytes", "omega_grid", "omega_argmin", "omega_grad",
           "omega_strerror", "omega_version", "omega_argmin_ex", "omega3_argmin_ex",
           "omega3_bands", "omega3_workspace_bytes",
           "omega3_grid", "omega3_argmin", "omega_chi_workspace_bytes", "omega_pair_chi",
           "omega3_chi_workspace_bytes", "omega3_pair_chi", "omega_q_wedge",
           "omega_lo_workspace_bytes", "omega_lo_grid", "omega_argmin_noalloc")


OMEGA_ETA_K, OMEGA_ETA_REL = 0, 1


class Model(ctypes.Structure):
    _fields_ = [("t1", ctypes.c_double), ("t2", ctypes.c_double),
                ("t3", ctypes.c_double), ("t4", ctypes.c_double),
                ("mu", ctypes.c_double), ("V", ctypes.c_double * 2),
                ("form", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Model3(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double * 12), ("eps0", ctypes.c_double),
                ("mu", ctypes.c_double), ("V", ctypes.c_double * 3),
                ("form", ctypes.c_int32), ("pad", ctypes.c_int32)]


class Point(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("T", ctypes.c_double),
                ("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32)]


class Launch(ctypes.Structure):
    """omega_launch: launch options of the _ex calls (results do not depend
    on them)."""
    _fields_ = [("sweep_blocks_per_cu", ctypes.c_int32), ("sweep_queues", ctypes.c_int32),
                ("sweep_start_event", ctypes.c_void_p), ("sweep_stop_event", ctypes.c_void_p),
                ("count_dev", ctypes.c_void_p)]


class OmegaError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = strerror(code) if _lib is not None else str(code)
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree libomega.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        # torch ships its own HIP runtime under the same soname; loading it
        # first makes libomega bind to that one runtime instance
        import torch  # noqa: F401
    except ImportError:
        pass
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python -m paper_1412_8754_amd.build")
    L = ctypes.CDLL(str(LIB_PATH))
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    mp, pp = ctypes.POINTER(Model), ctypes.POINTER(Point)
    L.omega_workspace_bytes.restype = sz
    L.omega_workspace_bytes.argtypes = [pp, i32, i32, i32, i32, i32, i32]
    L.omega_grid.restype = i32
    L.omega_grid.argtypes = [mp, pp, i32, vp, i32, vp, i32, i32, i32, vp, sz, vp, vp]
    L.omega_argmin.restype = i32
    L.omega_argmin.argtypes = [mp, pp, i32, vp, i32, vp, i32, i32, i32, ctypes.c_double,
                               vp, sz, vp, vp, vp, vp, vp]
    L.omega_grad.restype = i32
    L.omega_grad.argtypes = [mp, pp, i32, vp, vp, i32, vp, sz, vp, vp, vp, vp, vp]
    L.omega_strerror.restype = ctypes.c_char_p
    L.omega_strerror.argtypes = [i32]
    L.omega_version.restype = i32
    L.omega_version.argtypes = []
    lp = ctypes.POINTER(Launch)
    L.omega_argmin_ex.restype = i32
    L.omega_argmin_ex.argtypes = [mp, pp, i32, vp, i32, vp, i32, i32, i32, ctypes.c_double,
                                  vp, sz, vp, vp, vp, vp, lp, vp]
    L.omega_argmin_noalloc.restype = i32
    L.omega_argmin_noalloc.argtypes = [mp, pp, i32, vp, i32, vp, i32, i32, i32,
                                       ctypes.c_double, vp, vp, vp, vp, vp]
    m3 = ctypes.POINTER(Model3)
    L.omega3_bands.restype = i32
    L.omega3_bands.argtypes = [m3, i32, i32, vp, sz, vp, vp]
    L.omega3_workspace_bytes.restype = sz
    L.omega3_workspace_bytes.argtypes = [pp, i32, i32, i32, i32, i32]
    L.omega3_grid.restype = i32
    L.omega3_grid.argtypes = [m3, pp, i32, vp, i32, vp, i32, i32, i32, vp, sz, vp, vp]
    L.omega_chi_workspace_bytes.restype = sz
    L.omega_chi_workspace_bytes.argtypes = [pp, i32, i32, i32]
    L.omega_pair_chi.restype = i32
    L.omega_pair_chi.argtypes = [mp, pp, i32, vp, i32, i32, vp, sz, vp, vp]
    L.omega3_chi_workspace_bytes.restype = sz
    L.omega3_chi_workspace_bytes.argtypes = [pp, i32, i32, i32]
    L.omega3_pair_chi.restype = i32
    L.omega3_pair_chi.argtypes = [m3, pp, i32, vp, i32, i32, vp, sz, vp, vp]
    L.omega_q_wedge.restype = i32
    L.omega_q_wedge.argtypes = [i32, i32, vp, vp, i32]
    L.omega_lo_workspace_bytes.restype = sz
    L.omega_lo_workspace_bytes.argtypes = [pp, i32, i32, vp, i32, i32]
    L.omega_lo_grid.restype = i32
    L.omega_lo_grid.argtypes = [mp, pp, i32, vp, i32, vp, i32, i32, vp, sz, vp, vp]
    L.omega3_argmin.restype = i32
    L.omega3_argmin.argtypes = [m3, pp, i32, vp, i32, vp, i32, i32, i32, ctypes.c_double,
                                vp, sz, vp, vp, vp, vp, vp]
    L.omega3_argmin_ex.restype = i32
    L.omega3_argmin_ex.argtypes = [m3, pp, i32, vp, i32, vp, i32, i32, i32, ctypes.c_double,
                                   vp, sz, vp, vp, vp, vp, lp, vp]
    _lib = L
    return L


def strerror(code: int) -> str:
    return load().omega_strerror(code).decode()


def make_model(m) -> Model:
    if isinstance(m, Model):
        return m
    return Model(float(m["t1"]), float(m["t2"]), float(m["t3"]), float(m["t4"]),
                 float(m["mu"]), (ctypes.c_double * 2)(*[float(v) for v in m["V"]]),
                 int(m.get("form", OMEGA_ETA_K)), 0)


def make_model3(m) -> Model3:
    if isinstance(m, Model3):
        return m
    return Model3((ctypes.c_double * 12)(*[float(v) for v in m["t"]]), float(m["eps0"]),
                  float(m["mu"]), (ctypes.c_double * 3)(*[float(v) for v in m["V"]]),
                  int(m.get("form", OMEGA_ETA_K)), 0)


def make_points(pts):
    arr = (Point * len(pts))()
    for i, (h, T, Lx, Ly) in enumerate(pts):
        arr[i] = Point(float(h), float(T), int(Lx), int(Ly))
    return arr


def n_bands(bands: int) -> int:
    return int(bool(bands & 1)) + int(bool(bands & 2))


def n_bands3(bands: int) -> int:
    return int(bool(bands & 1)) + int(bool(bands & 2)) + int(bool(bands & 4))
