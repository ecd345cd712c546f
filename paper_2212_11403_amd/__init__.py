"""MI355X (gfx950) implementation of the Li & Stephens all-vs-all copying
model's forward/backward sweep, posterior decoding and PAC-likelihood
gradient, behind the C ABI of include/ls.h (libls.so).

The Python layer only marshals torch device tensors into that ABI; the
library must be built (``paper_2212_11403_amd.build.build()``) and there is
no CPU fallback.
"""

from ._lib import (LS_FP32, LS_FP32_F16STORE, LS_FP64, LS_MAX_TARGETS, LS_OK,
                   LS_WARN_NONFINITE, LsError, load)

__all__ = [
    "LS_FP32", "LS_FP32_F16STORE", "LS_FP64", "LS_MAX_TARGETS", "LS_OK", "LS_WARN_NONFINITE",
    "LsError", "load", "Model", "Table", "forward", "backward", "posterior_distance",
    "distance_symmetrise", "loglik_grad", "kernel_shape", "status_check", "decode",
    "PACLoglik", "RhoMap", "calc_rho", "rho_map_grad", "distance_matrices", "average_linkage",
    "average_linkage_noalloc", "standardise_rows",
]


def __getattr__(name):
    # the torch-facing API is imported on first use, so that importing the
    # package (e.g. to build it) does not pull in torch
    if name in ("Model", "Table", "forward", "backward", "posterior_distance",
                "distance_symmetrise", "loglik_grad", "kernel_shape", "status_check", "decode",
                "io_dtype", "prec_code", "calc_rho", "rho_map_grad", "distance_matrices",
                "average_linkage", "average_linkage_noalloc", "standardise_rows"):
        from . import api
        return getattr(api, name)
    if name in ("PACLoglik", "RhoMap"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
