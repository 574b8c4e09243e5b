"""ctypes binding of libsmnn.so (include/smnn.h).  Argument marshalling only:
every step of the solve runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmnn.so")

MODES = {"fp64": 0, "fp64r": 1, "fp32r": 2}

STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported order, chunk length or instance shape",
          3: "workspace or factor too small", 4: "HIP runtime error", 5: "wrong current device"}

Q_LEVELS, Q_CHUNK, Q_REFINE, Q_MODE, Q_CHUNK_UPPER, Q_INIT_POINTS, Q_TOP_LEVEL = 1, 2, 3, 4, 5, 6, 7


class SmnnError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__("%s: %s (status %d)" % (what, STATUS.get(status, "unknown"), status))
        self.status = status


class TraceRecord(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("level", ctypes.c_int32), ("rhs", ctypes.c_int32),
                ("out", ctypes.c_int32), ("ms", ctypes.c_float)]


KERNEL_NAMES = {1: "reduce0", 2: "reduceN", 3: "backsubN", 4: "backsub0", 5: "dw_reduce", 6: "info",
                7: "backsub_reduce0", 8: "top"}


class TuneResult(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("chunk_upper", ctypes.c_int32), ("block", ctypes.c_int32),
                ("max_blocks", ctypes.c_int32), ("ms", ctypes.c_float)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("n_init", ctypes.c_int32), ("n_inst", ctypes.c_int64),
                ("steps", ctypes.POINTER(ctypes.c_int64)), ("steps_uniform", ctypes.c_int64),
                ("mode", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("chunk_upper", ctypes.c_int32), ("block", ctypes.c_int32), ("max_blocks", ctypes.c_int32),
                ("init_points", ctypes.c_int32), ("variables", ctypes.c_int32), ("equations", ctypes.c_int32),
                ("row_weights", ctypes.c_int32)]


_lib = None


def lib():
    """Load libsmnn.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsmnn.so is not built (run: python -m paper_2410_06074_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.smnn_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
        L.smnn_plan_create.restype = ctypes.c_int
        L.smnn_plan_destroy.argtypes = [vp]
        L.smnn_plan_destroy.restype = ctypes.c_int
        L.smnn_plan_sizes.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(ctypes.c_int64)]
        L.smnn_plan_sizes.restype = ctypes.c_int
        L.smnn_plan_query.argtypes = [vp, ctypes.c_int32]
        L.smnn_plan_query.restype = ctypes.c_int64
        L.smnn_forward.argtypes = [vp] * 8 + [sz, vp, sz, vp, vp]
        L.smnn_forward.restype = ctypes.c_int
        L.smnn_forward_noalloc.argtypes = [vp] * 8 + [sz, vp, vp]
        L.smnn_forward_noalloc.restype = ctypes.c_int
        L.smnn_backward.argtypes = [vp] * 8 + [sz] + [vp] * 7 + [sz, vp, vp]
        L.smnn_backward.restype = ctypes.c_int
        L.smnn_trace_enable.argtypes = [vp, ctypes.c_int32]
        L.smnn_trace_enable.restype = ctypes.c_int
        L.smnn_trace_read.argtypes = [vp, ctypes.POINTER(TraceRecord), ctypes.c_int32]
        L.smnn_trace_read.restype = ctypes.c_int32
        L.smnn_autotune.argtypes = [ctypes.POINTER(PlanDesc)] + [vp] * 6 + [ctypes.c_int32, vp,
                                    ctypes.POINTER(TuneResult), ctypes.POINTER(TuneResult), ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_int32)]
        L.smnn_autotune.restype = ctypes.c_int
        L.smnn_status_string.argtypes = [ctypes.c_int]
        L.smnn_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != 0:
        raise SmnnError(status, what)
