"""ctypes declarations of the C ABI in include/acm.h (argument marshalling only).

Loading fails loudly when libacm.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libacm.so")

ACM_OK, ACM_NOT_CONVERGED = 0, 1
ACM_E_INVALID, ACM_E_UNSUPPORTED_SIZE, ACM_E_NOMEM, ACM_E_HIP, ACM_E_DIVERGED = -1, -2, -3, -4, -5
ACM_FP32, ACM_FP64 = 0, 1
KERNEL_KINDS = ["green", "local", "rhs", "y_inv", "y_fwd", "t_green", "t_local", "other"]
HIST_DOUBLES = 15


class acm_grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3)]


class acm_penalty(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double), ("b", C.c_double),
                ("phi", C.c_double * 3), ("tau", C.c_double * 3), ("psi_min", C.c_double * 3),
                ("adaptive", C.c_int32)]


class acm_opts(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_iter", C.c_int64), ("precision", C.c_int32),
                ("check_every", C.c_int32), ("warm_start", C.c_int32), ("use_graph", C.c_int32),
                ("profile", C.c_int32), ("history_cap", C.c_int32), ("pass_mode", C.c_int32),
                ("green_variant", C.c_int32), ("derivative", C.c_int32), ("step1_form", C.c_int32),
                ("transport_form", C.c_int32)]


class acm_stats(C.Structure):
    _fields_ = [("iters", C.c_int64), ("r_p", C.c_double * 3), ("r_d", C.c_double * 3),
                ("tol_p", C.c_double * 3), ("tol_d", C.c_double * 3), ("psi", C.c_double * 3),
                ("seconds", C.c_double), ("converged", C.c_int32), ("status", C.c_int32),
                ("kernel_ms", C.c_double * 8), ("kernel_calls", C.c_int64 * 8)]


class acm_fno_shape(C.Structure):
    _fields_ = [("channels", C.c_int32), ("hidden", C.c_int32), ("modes", C.c_int32),
                ("layers", C.c_int32)]


# name -> (restype, argtypes)
SIGNATURES = {
    "acm_default_penalty": (None, [C.POINTER(acm_penalty)]),
    "acm_default_opts": (None, [C.POINTER(acm_opts)]),
    "acm_last_error": (C.c_char_p, []),
    "acm_version": (C.c_int32, []),
    "acm_stokes_solve": (C.c_int, [C.POINTER(acm_grid), C.c_void_p, C.POINTER(C.c_double), C.c_double,
                                   C.POINTER(acm_penalty), C.POINTER(acm_opts), C.c_void_p, C.c_void_p,
                                   C.POINTER(acm_stats), C.POINTER(C.c_double), C.c_void_p]),
    "acm_stokes_solve_batched": (C.c_int, [C.c_int32, C.POINTER(acm_grid), C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_double), C.c_double, C.POINTER(acm_penalty),
                                           C.POINTER(acm_opts), C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_void_p), C.POINTER(acm_stats), C.c_void_p]),
    "acm_transport_step": (C.c_int, [C.POINTER(acm_grid), C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                     C.c_double, C.c_double, C.c_double, C.c_double,
                                     C.POINTER(C.c_double), C.c_double, C.c_int32,
                                     C.POINTER(acm_opts), C.c_void_p, C.POINTER(acm_stats), C.c_void_p]),
    "acm_effective_props": (C.c_int, [C.POINTER(acm_grid), C.c_int32, C.c_void_p, C.c_int32,
                                      C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p), C.c_void_p,
                                      C.c_double, C.c_double, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "acm_effective_props_noalloc": (C.c_int, [C.POINTER(acm_grid), C.c_int32, C.c_void_p, C.c_int32,
                                              C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p),
                                              C.c_void_p, C.c_double, C.c_double, C.POINTER(C.c_double),
                                              C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "acm_fno_param_count": (C.c_int64, [C.POINTER(acm_fno_shape)]),
    "acm_fno_workspace_bytes": (C.c_int64, [C.POINTER(acm_fno_shape), C.POINTER(acm_grid), C.c_int32,
                                            C.c_int32]),
    "acm_fno_forward": (C.c_int, [C.POINTER(acm_fno_shape), C.POINTER(acm_grid), C.c_int32, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p]),
    "acm_fno_backward": (C.c_int, [C.POINTER(acm_fno_shape), C.POINTER(acm_grid), C.c_int32, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "acm_fno_adam": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int64, C.c_double, C.c_double, C.c_double, C.c_double, C.c_void_p]),
    "acm_fno_to_bf16": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "acm_fno_mse": (C.c_int, [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                              C.c_void_p]),
    "acm_fft_r2c": (C.c_int, [C.POINTER(acm_grid), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "acm_fft_c2r": (C.c_int, [C.POINTER(acm_grid), C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
}

_lib = None


ABI_VERSION = 6  # must equal acm_version() of the loaded library


def load(path: str = LIB_PATH):
    """Load libacm.so and declare its entry points.  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is not built: run python -m paper_2312_15554_amd.build.  "
            "There is no CPU fallback.")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if lib.acm_version() != ABI_VERSION:
        raise RuntimeError(f"{path} has ABI version {lib.acm_version()}, these bindings expect "
                           f"{ABI_VERSION}: rebuild the library")
    _lib = lib
    return lib


class AcmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"acm status {status}: {msg}")
        self.status = status


def check(status: int) -> int:
    if status < 0:
        raise AcmError(status, load().acm_last_error().decode())
    return status
