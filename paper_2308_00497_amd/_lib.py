"""ctypes declarations of the C ABI in include/fft.h.

Argument marshalling only: every step of the transform runs in the HIP
library.  There is no fallback: if ``lib/libfft_mi355x.so`` is missing it is
built once with hipcc, and if that fails importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "lib", "libfft_mi355x.so")

FFT_LAYOUT_INTERLEAVED = 0
FFT_LAYOUT_SPLIT = 1
FFT_FORWARD = -1
FFT_INVERSE = 1
FFT_PRECISION_FP32 = 0
FFT_PRECISION_FP64 = 1

STATUS = {
    0: "FFT_OK",
    1: "FFT_ERR_INVALID_SIZE",
    2: "FFT_ERR_INVALID_ARG",
    3: "FFT_ERR_NULL_POINTER",
    4: "FFT_ERR_MISALIGNED",
    5: "FFT_ERR_ALLOC",
    6: "FFT_ERR_HIP",
    7: "FFT_ERR_NOT_SUPPORTED",
}

# every symbol include/fft.h declares
EXPORTS = [
    "fft_plan_create",
    "fft_plan_create_explicit",
    "fft_plan_create_ex",
    "fft_plan_create_real",
    "fft_plan_create_nd",
    "fft_execute",
    "fft_execute_backward",
    "fft_execute_no_alloc",
    "fft_no_alloc_scratch_bytes",
    "fft_plan_destroy",
    "fft_plan_create_ragged",
    "fft_plan_create_ragged_ex",
    "fft_plan_workspace_bytes",
    "fft_plan_set_workspace",
    "fft_plan_sizes",
    "fft_plan_describe",
    "fft_query_decomposition",
    "fft_copy_device",
    "fft_status_string",
    "fft_last_error_detail",
]


class FFTError(RuntimeError):
    """A non-OK fft_status from the library."""

    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        self.status = STATUS.get(code, f"status {code}")
        msg = f"{what}: {self.status}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.fft_plan_create.argtypes = [ctypes.POINTER(vp), i64, i64, ci, ci]
    lib.fft_plan_create_explicit.argtypes = [ctypes.POINTER(vp), i64, i64, ci, ci, ctypes.c_char_p]
    lib.fft_plan_create_ex.argtypes = [ctypes.POINTER(vp), i64, i64, ci, ci, ci, ctypes.c_char_p]
    lib.fft_plan_create_real.argtypes = [ctypes.POINTER(vp), i64, i64, ci, ci, ci, ctypes.c_char_p]
    lib.fft_plan_create_nd.argtypes = [ctypes.POINTER(vp), ci, ctypes.POINTER(i64), i64, ci, ci, ci]
    lib.fft_execute.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.fft_execute_backward.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.fft_execute_no_alloc.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.fft_no_alloc_scratch_bytes.argtypes = []
    lib.fft_plan_destroy.argtypes = [vp]
    lib.fft_plan_create_ragged.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64), i64, ci, ci]
    lib.fft_plan_create_ragged_ex.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(i64), i64, ci, ci, ctypes.c_char_p]
    lib.fft_plan_workspace_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    lib.fft_plan_set_workspace.argtypes = [vp, vp]
    lib.fft_plan_sizes.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
    lib.fft_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    lib.fft_query_decomposition.argtypes = [i64, ci, ci, ctypes.c_char_p, ctypes.c_size_t]
    lib.fft_copy_device.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.fft_status_string.argtypes = [ci]
    lib.fft_status_string.restype = ctypes.c_char_p
    lib.fft_last_error_detail.argtypes = []
    lib.fft_last_error_detail.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("fft_status_string", "fft_last_error_detail", "fft_no_alloc_scratch_bytes"):
            getattr(lib, name).restype = ci
    lib.fft_no_alloc_scratch_bytes.restype = ctypes.c_size_t
    return lib


def _open() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        from . import build as _build  # compile once; no other path exists
        _build.build()
    return _declare(ctypes.CDLL(LIB_PATH))


lib = _open()


def check(code: int, what: str) -> None:
    if code != 0:
        detail = lib.fft_last_error_detail()
        raise FFTError(code, what, detail.decode() if detail else "")
