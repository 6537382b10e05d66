"""ctypes loader for libols.so (the C ABI declared in include/ols.h).

Argument marshalling only: every step of the method runs in the HIP kernels.
There is no fallback: if the library is missing the import of an entry point
raises, naming the build command.
"""

from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libols.so")
EMU_PATH = os.path.join(_PKG, "lib", "libols_emu.so")

OLS_SUCCESS = 0
POST_NONE, POST_DERIVATIVE, POST_POWER = 0, 1, 2
STATUS_NAMES = {
    0: "OLS_SUCCESS",
    1: "OLS_ERROR_INVALID_VALUE",
    2: "OLS_ERROR_UNSUPPORTED",
    3: "OLS_ERROR_OUT_OF_MEMORY",
    4: "OLS_ERROR_HIP",
    5: "OLS_ERROR_INTERNAL",
}

# name -> (restype, argtypes), the exported symbols of include/ols.h
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_PI32 = ctypes.POINTER(ctypes.c_int32)
SIGNATURES = {
    "ols_plan": (_I32, [ctypes.POINTER(_P), _P, _I32, _I32, _I32, _P]),
    "ols_plan_ex": (_I32, [ctypes.POINTER(_P), _P, _I32, _I32, _I32, _I32, _P]),
    "ols_plan_update_filters": (_I32, [_P, _P, _P]),
    "ols_plan_set_hop": (_I32, [_P, _I32]),
    "ols_plan_set_stencil": (_I32, [_P, _I32, _I32, _I32, _P]),
    "ols_plan_get_info": (_I32, [_P, _PI32, _PI32, _PI32, _PI32, _PI32]),
    "ols_plan_get_spectra": (_I32, [_P, _P, _P]),
    "ols_plan_get_launch": (_I32, [_P, _PI32, _PI32, _PI32]),
    "ols_plan_set_tiling": (_I32, [_P, _I32, _I32]),
    "ols_plan_get_fft_length": (_I32, [_P, _PI32]),
    "ols_batched_workspace_size": (_I32, [_P, _I32, ctypes.POINTER(ctypes.c_size_t)]),
    "ols_plan_get_tiling": (_I32, [_P, _PI32, _PI32, _PI32]),
    "ols_forward": (_I32, [_P, _P, _I64, _P, _P]),
    "ols_plan_destroy": (_I32, [_P]),
    "ols_backward": (_I32, [_P, _P, _I64, _P, _P, _P, _P]),
    "ols_backward_static": (_I32, [_P, _P, _I64, _P, _P, _P, _P]),
    "ols_plan_reserve_backward": (_I32, [_P]),
    "ols_batch_plan": (_I32, [ctypes.POINTER(_P), _P, _I32, _P]),
    "ols_batch_run": (_I32, [_P, _P]),
    "ols_batched": (_I32, [_P, _I32, _P, ctypes.c_size_t, _P]),
    "ols_batched_status": (_I32, [_P, _P, _PI32, _PI32]),
    "ols_batch_get_info": (_I32, [_P, ctypes.POINTER(_I64), _PI32, _PI32]),
    "ols_batch_get_item": (_I32, [_P, _I32, _PI32, _PI32, _PI32]),
    "ols_batch_destroy": (_I32, [_P]),
    "ols_status_string": (ctypes.c_char_p, [_I32]),
    "ols_last_error": (ctypes.c_char_p, []),
    "ols_calibration_copy": (_I32, [_P, _P, ctypes.c_size_t, _P]),
}


class BatchItem(ctypes.Structure):
    """ols_batch_item_t of include/ols.h."""
    _fields_ = [("s", ctypes.c_void_p), ("N_s", ctypes.c_int64), ("h", ctypes.c_void_p), ("K", ctypes.c_int32),
                ("M", ctypes.c_int32), ("N", ctypes.c_int32), ("y", ctypes.c_void_p)]


class OLSError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} {detail}".strip())


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libols.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1910_01972_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, where: str) -> None:
    if status != OLS_SUCCESS:
        detail = lib().ols_last_error().decode(errors="replace")
        raise OLSError(status, where, detail)
