"""MI355X (gfx950) implementation of the free-energy search of Januszewski,
Ptok, Crivelli & Gardas, "GPU-based acceleration of free energy calculations
in solid state physics": the FF free energy Omega(Delta, Q; h, T, mu) of the
two-band iron-pnictide model over parameter grids, its minima (Algorithm 1)
and its gradient.

The computation lives in libomega.so (HIP kernels behind the C interface of
include/omega.h); `api` marshals torch tensors into it.
"""
from ._abi import (OMEGA_BAND_BOTH, OMEGA_BAND_MINUS, OMEGA_BAND_PLUS,  # noqa: F401
                   OMEGA_ETA_K, OMEGA_ETA_REL, OMEGA_FP32_COMP, OMEGA_FP64, OmegaError)

__all__ = ["OMEGA_BAND_BOTH", "OMEGA_BAND_MINUS", "OMEGA_BAND_PLUS", "OMEGA_ETA_K",
           "OMEGA_ETA_REL", "OMEGA_FP32_COMP", "OMEGA_FP64", "OmegaError"]
