"""ctypes view of libtsm2x.so (the C ABI of include/tsm2x.h).

Argument marshalling only: every product runs in the library's HIP kernels.
If the library has not been built, loading raises immediately; there is no
fallback implementation."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# TSM2X_LIBRARY may point at another build of the same library
LIB_PATH = os.environ.get("TSM2X_LIBRARY") or os.path.join(HERE, "libtsm2x.so")

F64, F32, BF16, F16, BF16_SPLIT, F16_SPLIT = range(6)
OP_TSM2R, OP_TSM2L, OP_GRAD_A, OP_GRAD_B, OP_TSM2R_ROWMAJOR, OP_KMEANS = range(6)

_lock = threading.Lock()
_lib = None


class TSMError(RuntimeError):
    def __init__(self, fn: str, code: int, lib):
        msg = lib.tsm2x_error_string(code).decode()
        if code == 2:
            msg += ": " + lib.tsm2x_last_hip_error().decode()
        super().__init__("%s returned %d (%s)" % (fn, code, msg))
        self.code = code


def lib():
    """The loaded library (raises if libtsm2x.so is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "libtsm2x.so is not built (run paper_2002_03258_amd/build.py "
                    "or __graft_entry__.build()); there is no fallback path")
            L = ctypes.CDLL(LIB_PATH)
            i64, vp, i32, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
            mm = [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, vp]
            L.tsm2r.argtypes = mm
            L.tsm2l.argtypes = mm
            ex = [i32, i32, i64, i64, i64, vp, i64, vp, i64, ctypes.c_double, vp, i64, i32, vp,
                  sz, vp]
            L.tsm2r_ex.argtypes = ex
            L.tsm2l_ex.argtypes = ex
            L.tsm2x_gemm.argtypes = ex
            L.tsm_grad_a.argtypes = mm
            L.tsm_grad_b.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, vp, sz, vp]
            L.tsm2x_split.argtypes = [i64, i64, vp, i64, vp, vp, i64, i32, vp]
            L.tsm2l_backward.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp, i64, vp, i64,
                                         i32, vp, sz, vp]
            L.tsm2l_backward_noalloc.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64, vp,
                                                 i64, vp, i64, i32, vp]
            L.tsm2l_backward_noalloc.restype = i32
            L.tsm_kmeans_assign.argtypes = [i64, i64, i64, vp, i64, i32, vp, i64, vp, vp, i32, vp,
                                            sz, vp]
            L.tsm2x_workspace_size.argtypes = [i32, i64, i64, i64, i32]
            L.tsm2x_workspace_size.restype = sz
            L.tsm2x_kernel_name.argtypes = [i32, i64, i64, i64, i32]
            L.tsm2x_kernel_name.restype = ctypes.c_char_p
            pi, p64 = ctypes.POINTER(i32), ctypes.POINTER(i64)
            L.tsm2x_tsm2r_plan.argtypes = [i64, i64, i64, i32, pi, pi, p64, pi, pi, pi]
            L.tsm2x_tsm2r_pin.argtypes = [i64, i64, i64, i32, i32, i32]
            L.tsm2x_error_string.argtypes = [i32]
            L.tsm2x_error_string.restype = ctypes.c_char_p
            L.tsm2x_last_hip_error.argtypes = []
            L.tsm2x_last_hip_error.restype = ctypes.c_char_p
            L.tsm2x_version.argtypes = []
            L.tsm2x_finalize.argtypes = []
            L.tsm2x_finalize.restype = None
            for f in ("tsm2x_timing_start", "tsm2x_timing_stop", "tsm2x_timing_tag",
                      "tsm2x_timing_collect"):
                getattr(L, f).argtypes = [i32] if f == "tsm2x_timing_tag" else []
                getattr(L, f).restype = i32
            L.tsm2x_timing_row.argtypes = [i32, ctypes.POINTER(ctypes.c_char_p), pi, p64,
                                           ctypes.POINTER(ctypes.c_double)]
            L.tsm2x_timing_row.restype = i32
            L.tsm2x_probe_stream.argtypes = [i32, vp, vp, i64, i64, vp]
            L.tsm2x_probe_stream.restype = i32
            L.tsm2x_probe_tiles.argtypes = [i64, i32, i32, vp, i64, vp, i64, vp, i64, i32, i64, vp]
            L.tsm2x_probe_tiles.restype = i32
            for f in ("tsm2r", "tsm2l", "tsm2r_ex", "tsm2l_ex", "tsm2x_gemm", "tsm_grad_a",
                      "tsm_grad_b",
                      "tsm2l_backward", "tsm2x_split", "tsm2x_version", "tsm2x_tsm2r_plan",
                      "tsm_kmeans_assign",
                      "tsm2x_tsm2r_pin"):
                getattr(L, f).restype = i32
            _lib = L
    return _lib


def call(fn: str, *args) -> None:
    L = lib()
    rc = getattr(L, fn)(*args)
    if rc != 0:
        raise TSMError(fn, rc, L)


EXPORTS = ("tsm2r", "tsm2r_ex", "tsm2l", "tsm2l_ex", "tsm2x_gemm", "tsm_grad_a", "tsm_grad_b",
           "tsm2l_backward", "tsm2l_backward_noalloc", "tsm_kmeans_assign",
           "tsm2x_split",
           "tsm2x_workspace_size", "tsm2x_kernel_name", "tsm2x_tsm2r_plan", "tsm2x_tsm2r_pin",
           "tsm2x_timing_start", "tsm2x_timing_stop", "tsm2x_timing_tag", "tsm2x_timing_collect",
           "tsm2x_timing_row", "tsm2x_probe_stream", "tsm2x_probe_tiles",
           "tsm2x_error_string", "tsm2x_last_hip_error",
           "tsm2x_version", "tsm2x_finalize")
