"""ctypes view of libmecuco.so (the C ABI declared in include/mecuco.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmecuco.so")

# constants mirrored from include/mecuco.h
MC_OK, MC_EINVAL, MC_ESHAPE, MC_EPRECISION, MC_EWORKSPACE, MC_ELAUNCH, MC_ENUMERIC, MC_EDEVICE, MC_ESCRATCH = range(9)
MC_NOALLOC_SCRATCH_BYTES = 64 << 20
MC_FP32, MC_BF16, MC_FP8, MC_FP64 = 0, 1, 2, 3
MC_FAST_FP64_KMAX = 28
MC_FAST_PAPER, MC_FAST_HAAR = 0, 1
MC_INCLUDE_SELF, MC_STRICT = 1, 2
MC_PF_NONFINITE, MC_PF_DEGENERATE, MC_PF_RANK_DEFICIENT = 1, 2, 4
MC_PF_JACOBI_MAXSWEEPS, MC_PF_KNN_AMBIGUOUS, MC_PF_KNN_UNCERTIFIED = 8, 16, 32
MC_PF_EIGEN_FP64 = 64
MC_PF_PRECISION_LIMIT = 128
MC_OP_KNN, MC_OP_FAST, MC_OP_EXACT, MC_OP_BACKWARD, MC_OP_NORMALIZE = 0, 1, 2, 3, 4
MC_KMAX = 32

EXPORTS = ("mc_knn", "mc_curvature_fast", "mc_curvature_exact", "mc_curvature_backward",
           "mc_curvature_fast_noalloc", "mc_normalize_minmax",
           "mc_workspace_bytes", "mc_status_string", "mc_version", "mc_timing_enable",
           "mc_timing_read", "mc_stage_name")
MC_STAGE_COUNT = 14
CURV_STAGES = ("curv_fast", "curv_gram", "curv_eigen", "curv_range")

_lib = None


class MecucoError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: status {status}: {status_string(status)}")


def lib() -> ctypes.CDLL:
    """The loaded library (loaded on first use)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2606_06329_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, u32, vp, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_size_t
    f32 = ctypes.c_float
    L.mc_knn.argtypes = [vp, i64, i64, i64, i32, i32, i32, u32, vp, vp, vp, vp, sz, vp]
    L.mc_knn.restype = ctypes.c_int
    L.mc_curvature_fast.argtypes = [vp, i64, i64, i64, vp, i32, i32, i32, u32, vp, vp, vp, sz, vp]
    L.mc_curvature_fast.restype = ctypes.c_int
    L.mc_curvature_fast_noalloc.argtypes = [vp, i64, i64, i64, vp, i32, i32, i32, u32, vp, vp, vp]
    L.mc_curvature_fast_noalloc.restype = ctypes.c_int
    L.mc_curvature_exact.argtypes = [vp, i64, i64, i64, vp, i32, i32, u32, vp, vp, vp, sz, vp]
    L.mc_curvature_exact.restype = ctypes.c_int
    L.mc_curvature_backward.argtypes = [vp, i64, i64, i64, vp, i32, i32, vp, f32, vp, vp, sz, vp]
    L.mc_curvature_backward.restype = ctypes.c_int
    L.mc_normalize_minmax.argtypes = [vp, i64, vp, vp, sz, vp]
    L.mc_normalize_minmax.restype = ctypes.c_int
    L.mc_workspace_bytes.argtypes = [i32, i64, i64, i32, i32, i32]
    L.mc_workspace_bytes.restype = sz
    L.mc_status_string.argtypes = [ctypes.c_int]
    L.mc_status_string.restype = ctypes.c_char_p
    L.mc_version.argtypes = []
    L.mc_version.restype = ctypes.c_int
    L.mc_timing_enable.argtypes = [ctypes.c_int]
    L.mc_timing_enable.restype = ctypes.c_int
    L.mc_timing_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.mc_timing_read.restype = ctypes.c_int
    L.mc_stage_name.argtypes = [i32]
    L.mc_stage_name.restype = ctypes.c_char_p
    _lib = L
    return L


def status_string(status: int) -> str:
    return lib().mc_status_string(int(status)).decode()


def check(status: int, where: str) -> None:
    if status != MC_OK:
        raise MecucoError(status, where)


def timing_enable(on: bool) -> None:
    check(lib().mc_timing_enable(1 if on else 0), "mc_timing_enable")


def timing_read() -> dict:
    """{stage name: (total ms, launches)} since the previous read; synchronises the events."""
    out = {}
    for st in range(MC_STAGE_COUNT):
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int64(0)
        check(lib().mc_timing_read(st, ctypes.byref(ms), ctypes.byref(cnt)), "mc_timing_read")
        if cnt.value:
            out[lib().mc_stage_name(st).decode()] = (ms.value, cnt.value)
    return out
