"""ctypes binding of libwstack.so: argument marshalling only.

Every computation happens in the HIP library; this module only loads it,
declares the C signatures of include/wstack.h and turns non-zero statuses
into exceptions.  There is no fallback: if the library is missing or fails
to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwstack.so")

WS_OK = 0
WS_INVALID_ARG = -1
WS_UNSUPPORTED_SIZE = -2
WS_WORKSPACE_TOO_SMALL = -3
WS_HIP_ERROR = -4
WS_BAD_STATE = -5
WS_FP32 = 0
WS_FP64 = 1
WS_KERNEL_GAUSS = 0
WS_KERNEL_ES = 1
WS_BINNING_AUTO = 0
WS_BINNING_PARTITION = 1
WS_BINNING_HASHED = 2
WS_NOALLOC_SCRATCH_BYTES = 64 << 20


class WStackError(RuntimeError):
    def __init__(self, status: int, func: str, message: str):
        super().__init__(f"{func}: {message} (status {status})")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("nu", C.c_int32), ("nv", C.c_int32), ("nw", C.c_int32),
        ("fov_l", C.c_double), ("fov_m", C.c_double),
        ("w_min", C.c_double), ("w_max", C.c_double),
        ("support", C.c_int32), ("sigma", C.c_double),
        ("precision", C.c_int32), ("tile", C.c_int32), ("chunk", C.c_int32),
        ("kernel", C.c_int32), ("beta", C.c_double), ("correct", C.c_int32),
        ("binning", C.c_int32),
    ]


_P = C.c_void_p
_SIGS = {
    "ws_validate_params": (C.c_int32, [C.POINTER(Params)]),
    "ws_workspace_bytes": (C.c_int32, [C.POINTER(Params), C.c_int64,
                                       C.POINTER(C.c_size_t),
                                       C.POINTER(C.c_size_t)]),
    "ws_kernel_transform": (C.c_int32, [C.POINTER(Params), C.c_int64, _P, _P,
                                        _P]),
    "ws_grid_init": (C.c_int32, [C.POINTER(Params), C.c_int64, _P, C.c_size_t,
                                 _P, C.c_size_t, _P, C.POINTER(_P)]),
    "ws_grid_visibilities": (C.c_int32, [_P, C.c_int64, _P, _P, _P, _P]),
    "ws_fft_planes": (C.c_int32, [_P, C.c_int32]),
    "ws_wcorrect_accumulate": (C.c_int32, [_P, _P]),
    "ws_image_accumulate": (C.c_int32, [_P, _P]),
    "ws_grid_image": (C.c_int32, [_P, C.c_int64, _P, _P, _P, _P, _P]),
    "ws_tile_stats": (C.c_int32, [_P, _P]),
    "ws_grid_rows": (C.c_int32, [_P, C.c_int64, C.c_int32, C.c_int32, _P,
                                 _P, _P, _P, _P, _P]),
    "ws_grid_image_rows": (C.c_int32, [_P, C.c_int64, C.c_int32, C.c_int32,
                                       _P, _P, _P, _P, _P, _P, _P]),
    "ws_dirty_beam": (C.c_int32, [_P, C.c_int64, _P, _P, _P, _P, _P]),
    "ws_residual_image": (C.c_int32, [_P, C.c_int64, _P, _P, _P, _P, _P, _P,
                                      _P, _P]),
    "ws_clean_minor": (C.c_int32, [_P, _P, _P, _P, C.c_int32, C.c_double,
                                   C.c_double, _P, _P]),
    "ws_degrid": (C.c_int32, [_P, _P, C.c_int32, C.c_int64, _P, _P, _P]),
    "ws_grid_image_noalloc": (C.c_int32, [C.POINTER(Params), C.c_int64, _P,
                                          _P, _P, _P, _P, _P]),
    "ws_plan_reset": (C.c_int32, [_P]),
    "ws_set_stream": (C.c_int32, [_P, _P]),
    "ws_sync": (C.c_int32, [_P]),
    "ws_set_profiling": (C.c_int32, [_P, C.c_int32]),
    "ws_kernel_times": (C.c_int32, [_P, C.c_int32, C.POINTER(C.c_char_p),
                                    C.POINTER(C.c_double),
                                    C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int32), C.c_int32]),
    "ws_batch_workspace_bytes": (C.c_int32, [C.c_int32,
                                             C.POINTER(C.c_size_t)]),
    "ws_batch_create": (C.c_int32, [C.c_int32, C.POINTER(_P), _P,
                                    C.c_size_t, C.POINTER(_P)]),
    "ws_batch_image": (C.c_int32, [_P, C.POINTER(C.c_int64), C.POINTER(_P),
                                   C.POINTER(_P), C.POINTER(_P),
                                   C.POINTER(_P)]),
    "ws_batch_capture": (C.c_int32, [_P, C.POINTER(C.c_int64),
                                     C.POINTER(_P), C.POINTER(_P),
                                     C.POINTER(_P), C.POINTER(_P)]),
    "ws_batch_replay": (C.c_int32, [_P]),
    "ws_batch_destroy": (None, [_P]),
    "ws_plan_destroy": (None, [_P]),
    "ws_status_string": (C.c_char_p, [C.c_int32]),
    "ws_last_error": (C.c_char_p, []),
}

_lib = None


def lib() -> C.CDLL:
    """Load libwstack.so once; raise if it is absent or incomplete."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} not found: build it with "
                "`python -m paper_2301_06061_amd.build` (no fallback exists)")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(status: int, func: str) -> None:
    if status != WS_OK:
        msg = lib().ws_last_error().decode(errors="replace")
        raise WStackError(status, func, msg)


def call(name: str, *args) -> int:
    st = getattr(lib(), name)(*args)
    check(st, name)
    return st


def exported_symbols() -> list:
    return list(_SIGS)
