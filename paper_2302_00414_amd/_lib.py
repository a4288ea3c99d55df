"""ctypes binding of ``libnfft_mi355x.so`` (declarations of include/nfft.h).

Argument marshalling only. The library must have been built in-tree
(``python -m paper_2302_00414_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnfft_mi355x.so")

NFFT_OK, NFFT_EINVAL, NFFT_ENOMEM, NFFT_EDEVICE, NFFT_ESTATE, NFFT_EUNSUPPORTED = range(6)
NFFT_F64, NFFT_F32 = 0, 1
NFFT_STAGES = 8
(NFFT_TUNE_TILE_EDGE, NFFT_TUNE_ITEM_NODES, NFFT_TUNE_SPREAD_THREADS, NFFT_TUNE_RHS_PER_GROUP,
 NFFT_TUNE_FFT_MIN_WG, NFFT_TUNE_SPREAD_PLANES, NFFT_TUNE_SPREAD_MODE) = range(7)
NFFT_TUNE_COUNT = 7

EXPORTS = (
    "nfft_plan", "nfft_plan_tuned", "nfft_plan_autotune", "nfft_get_tuning", "nfft_set_tuning",
    "nfft_plan_clone",
    "nfft_set_weights", "nfft_adjoint", "nfft_adjoint_scratch", "nfft_forward", "nfft_refine",
    "nfft_weights",
    "nfft_weights_ex",
    "nfft_bopt_build",
    "nfft_bopt_adjoint", "nfft_bopt_inverse_adjoint", "nfft_bopt_get", "nfft_destroy",
    "nfft_footprint", "nfft_strerror", "nfft_last_error", "nfft_plan_info",
    "nfft_permutation", "nfft_set_profiling", "nfft_stage_times",
)

_lib = None


class NfftError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{status} ({_strerror(status)}): {detail}")


def _strerror(status: int) -> str:
    return load().nfft_strerror(status).decode()


def load() -> ctypes.CDLL:
    """Load the library once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_00414_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.nfft_plan.argtypes = [ctypes.POINTER(vp), i32, i32, dbl, i32, i64, vp, i32, i32, vp]
    lib.nfft_plan.restype = i32
    lib.nfft_plan_tuned.argtypes = [ctypes.POINTER(vp), i32, i32, dbl, i32, i64, vp, i32, i32,
                                    ctypes.POINTER(i32), i32, vp]
    lib.nfft_plan_tuned.restype = i32
    lib.nfft_plan_autotune.argtypes = [ctypes.POINTER(vp), i32, i32, dbl, i32, i64, vp, i32, i32, i32,
                                       ctypes.POINTER(dbl), vp]
    lib.nfft_plan_autotune.restype = i32
    lib.nfft_get_tuning.argtypes = [vp, ctypes.POINTER(i32), i32]
    lib.nfft_get_tuning.restype = i32
    lib.nfft_set_tuning.argtypes = [vp, i32, i32]
    lib.nfft_set_tuning.restype = i32
    lib.nfft_plan_clone.argtypes = [vp, i32, ctypes.POINTER(vp), vp]
    lib.nfft_plan_clone.restype = i32
    lib.nfft_set_weights.argtypes = [vp, vp, vp]
    lib.nfft_set_weights.restype = i32
    lib.nfft_adjoint.argtypes = [vp, vp, vp, i32, vp]
    lib.nfft_adjoint.restype = i32
    lib.nfft_adjoint_scratch.argtypes = [vp, vp, vp, i32, vp]
    lib.nfft_adjoint_scratch.restype = i32
    lib.nfft_forward.argtypes = [vp, vp, vp, i32, vp]
    lib.nfft_forward.restype = i32
    lib.nfft_refine.argtypes = [vp, vp, vp, i32, i32, ctypes.POINTER(dbl), vp]
    lib.nfft_refine.restype = i32
    lib.nfft_weights.argtypes = [i32, i32, dbl, i32, i64, vp, dbl, i32, vp, ctypes.POINTER(dbl), vp]
    lib.nfft_weights.restype = i32
    lib.nfft_weights_ex.argtypes = [i32, i32, dbl, i32, i64, vp, i32, dbl, i32, vp,
                                    ctypes.POINTER(dbl), vp]
    lib.nfft_weights_ex.restype = i32
    lib.nfft_bopt_build.argtypes = [vp, vp, ctypes.POINTER(dbl), vp]
    lib.nfft_bopt_build.restype = i32
    lib.nfft_bopt_adjoint.argtypes = [vp, vp, vp, i32, vp]
    lib.nfft_bopt_adjoint.restype = i32
    lib.nfft_bopt_inverse_adjoint.argtypes = [vp, vp, vp, i32, vp]
    lib.nfft_bopt_inverse_adjoint.restype = i32
    lib.nfft_bopt_get.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(dbl)]
    lib.nfft_bopt_get.restype = i32
    lib.nfft_destroy.argtypes = [vp]
    lib.nfft_destroy.restype = i32
    lib.nfft_footprint.argtypes = [i32, i32, dbl, i32, i64, i32, i32]
    lib.nfft_footprint.restype = i64
    lib.nfft_strerror.argtypes = [i32]
    lib.nfft_strerror.restype = ctypes.c_char_p
    lib.nfft_last_error.argtypes = [vp]
    lib.nfft_last_error.restype = ctypes.c_char_p
    lib.nfft_plan_info.argtypes = [vp, ctypes.POINTER(i64), i32]
    lib.nfft_plan_info.restype = i32
    lib.nfft_permutation.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    lib.nfft_permutation.restype = i32
    lib.nfft_set_profiling.argtypes = [vp, i32]
    lib.nfft_set_profiling.restype = i32
    lib.nfft_stage_times.argtypes = [vp, ctypes.POINTER(dbl), i32, i32]
    lib.nfft_stage_times.restype = i32
    _lib = lib
    return lib


def check(status: int, plan=None) -> None:
    if status != NFFT_OK:
        detail = load().nfft_last_error(plan).decode(errors="replace")
        raise NfftError(status, detail)
