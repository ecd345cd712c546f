"""ctypes declarations of libls (include/ls.h). Argument marshalling only."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libls.so")

LS_OK = 0
LS_ERR_ARG = 1
LS_ERR_SHAPE = 2
LS_ERR_STATE = 3
LS_ERR_UNSUPPORTED = 4
LS_ERR_DEVICE = 5
LS_ERR_WORKSPACE = 6
LS_ERR_SCRATCH = 7
LS_WARN_NONFINITE = 16

LS_FP64 = 0
LS_FP32 = 1
LS_FP32_F16STORE = 2

LS_FLAG_NONFINITE = 1
LS_FLAG_BAD_RECIPIENT = 2
LS_MAX_TARGETS = 256

# every symbol include/ls.h declares
EXPORTED = [
    "ls_model_workspace_bytes", "ls_model_init", "ls_table_init", "ls_table_copy",
    "ls_forward", "ls_backward", "ls_posterior_distance", "ls_distance_symmetrise",
    "ls_loglik_grad", "ls_loglik_grad_workspace_bytes", "ls_status_check",
    "ls_kernel_shape", "ls_status_string", "ls_version", "ls_calc_rho", "ls_rho_map_grad",
    "ls_loglik_checkpoint", "ls_loglik_grad_adjoint", "ls_average_linkage",
    "ls_average_linkage_workspace_bytes", "ls_average_linkage_noalloc", "ls_standardise_rows",
]


class LsModel(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_void_p),
        ("stride_words", ctypes.c_int64),
        ("N", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("rho", ctypes.c_void_p),
        ("mu", ctypes.c_double),
        ("hash", ctypes.c_uint64),
        ("Hr", ctypes.c_void_p),
        ("hr_stride", ctypes.c_int64),
        ("nf", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("mu_vec", ctypes.c_void_p),
        ("prior", ctypes.c_void_p),
    ]


class LsTable(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_void_p),
        ("log_scale", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("recipients", ctypes.c_void_p),
        ("R", ctypes.c_int32),
        ("l", ctypes.c_int32),
        ("direction", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("model_hash", ctypes.c_uint64),
    ]


class LsError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} (code {code})")


_lib = None


def load():
    """Load libls.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with paper_2212_11403_amd.build.build() "
            "(the GPU path has no CPU fallback)")
    # The binding hands torch device memory and streams to the library, so
    # both must use one HIP runtime. torch ships its own libamdhip64.so.7;
    # once it is loaded it also satisfies libls.so's dependency. Opened
    # first, libls.so would map the system runtime and torch would then map
    # its own beside it, and pointers from one are invalid in the other.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, SZ, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                               ctypes.c_size_t, ctypes.c_double)
    M = ctypes.POINTER(LsModel)
    T = ctypes.POINTER(LsTable)
    sig = {
        "ls_model_workspace_bytes": (SZ, [I32, I32]),
        "ls_model_init": (ctypes.c_int, [M, P, SZ, P]),
        "ls_table_init": (ctypes.c_int, [T, I32, ctypes.c_int, P, P, P, P, I32, P]),
        "ls_table_copy": (ctypes.c_int, [T, T, I32, P]),
        "ls_forward": (ctypes.c_int, [T, M, I32, P, I32, P, P, P, I64, I64, P]),
        "ls_backward": (ctypes.c_int, [T, M, I32, P, I32, P, P]),
        "ls_posterior_distance": (ctypes.c_int, [T, T, M, P, P, P]),
        "ls_distance_symmetrise": (ctypes.c_int, [P, P, I32, I32, ctypes.c_int, P]),
        "ls_loglik_grad": (ctypes.c_int, [M, P, I32, ctypes.c_int, P, P, P, P, P, SZ, P]),
        "ls_loglik_grad_workspace_bytes": (SZ, [M, I32, ctypes.c_int]),
        "ls_loglik_checkpoint": (ctypes.c_int, [M, P, I32, ctypes.c_int, P, P, P, SZ, P]),
        "ls_average_linkage_workspace_bytes": (SZ, [I32, I32, ctypes.c_int]),
        "ls_average_linkage": (ctypes.c_int, [P, I32, I32, ctypes.c_int, P, P, P, SZ, P]),
        "ls_average_linkage_noalloc": (ctypes.c_int, [P, I32, I32, ctypes.c_int, P, P, P]),
        "ls_standardise_rows": (ctypes.c_int, [P, P, I32, I32, I32, I64, I64, ctypes.c_int, P]),
        "ls_loglik_grad_adjoint": (ctypes.c_int, [M, P, I32, ctypes.c_int, P, P, P, SZ, P]),
        "ls_status_check": (ctypes.c_int, [P, I32, P]),
        "ls_kernel_shape": (ctypes.c_int, [I32, ctypes.c_int, I32, ctypes.POINTER(I32),
                                           ctypes.POINTER(I32)]),
        "ls_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "ls_version": (ctypes.c_char_p, []),
        "ls_calc_rho": (ctypes.c_int, [P, I32, D, D, P, P]),
        "ls_rho_map_grad": (ctypes.c_int, [P, I32, D, D, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(code: int) -> str:
    try:
        return load().ls_status_string(code).decode()
    except Exception:  # library not loadable: still format the error
        return "status"


def check(code: int, what: str):
    if code != LS_OK:
        raise LsError(code, what)
