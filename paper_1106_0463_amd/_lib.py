"""ctypes declarations of the C ABI in ``include/lc.h`` (argument marshalling
only; every step of the computation runs in the HIP library).

The library ``liblc.so`` is built in-tree by :mod:`paper_1106_0463_amd.build`.
Loading fails loudly when it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblc.so")

LC_OK, LC_ERR_INVALID, LC_ERR_NOMEM, LC_ERR_HIP, LC_ERR_UNSUPPORTED, LC_ERR_INTERNAL = range(6)
LC_FP64, LC_FP32_QUAD = 0, 1
GEMM_MODES = {"fp64": 0, "bf16x3": 1, "bf16x6": 2, "fp16x3": 3, "fp16x1": 4}
PRECISIONS = {"fp64": LC_FP64, "fp32": LC_FP32_QUAD}


class PlanDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("precision", C.c_int32), ("N", C.c_int64),
                ("M", C.c_int64), ("M_eff", C.c_int64), ("H", C.c_int64),
                ("Q", C.c_int32), ("B", C.c_int32), ("samples", C.c_int64),
                ("sample_bytes", C.c_int64), ("workspace_bytes", C.c_int64)]


class AbelRule(C.Structure):
    _fields_ = [("q", C.c_int32), ("q_max", C.c_int32), ("band", C.c_double), ("nbreak", C.c_int32),
                ("breaks", C.POINTER(C.c_double)), ("grade_ratio", C.c_double),
                ("grade_levels", C.c_int32)]


# (name, restype, argtypes) for every symbol the header declares
_vp, _i32, _i64 = C.c_void_p, C.c_int32, C.c_int64
_pi64, _pi32 = C.POINTER(C.c_int64), C.POINTER(C.c_int32)
SIGNATURES = [
    ("lc_grid_size", C.c_int, [_i64, _pi64]),
    ("lc_plan", C.c_int, [_i64, _i64, _i32, C.c_int, C.POINTER(_vp)]),
    ("lc_plan_adaptive", C.c_int, [_i64, _i64, C.POINTER(AbelRule), C.c_int, C.POINTER(_vp)]),
    ("lc_plan_2d", C.c_int, [_i64, _i64, _i32, C.c_int, C.POINTER(_vp)]),
    ("lc_execute_2d", C.c_int, [_vp, _vp, _vp, _vp]),
    ("lc_plan_info", C.c_int, [_vp, C.POINTER(PlanDesc)]),
    ("lc_plan_nodes", C.c_int, [_vp, C.POINTER(_vp), _pi64, _pi32]),
    ("lc_plan_nodes_complement", C.c_int, [_vp, _vp, _vp]),
    ("lc_execute", C.c_int, [_vp, _vp, _vp, _vp]),
    ("lc_execute_noalloc", C.c_int, [_vp, _vp, _vp, _vp]),
    ("lc_plan_batch", C.c_int, [_i32, _pi64, _pi64, _pi32, C.POINTER(C.c_int), C.POINTER(_vp)]),
    ("lc_plan_batch_rules", C.c_int, [_i32, _pi64, _pi64, C.POINTER(AbelRule), C.POINTER(C.c_int),
                                      C.POINTER(_vp)]),
    ("lc_plan_batch_offsets", C.c_int, [_vp, _pi64, _pi64, _pi64]),
    ("lc_execute_batch", C.c_int, [_vp, _vp, _vp, _vp]),
    ("lc_plan_gemm", C.c_int, [_i32, _i64, _i64, C.c_int, C.POINTER(_vp)]),
    ("lc_plan_legendre_matrix", C.c_int, [_i32, _i64, _i64, C.c_int, C.POINTER(_vp)]),
    ("lc_execute_gemm", C.c_int, [_vp, _vp, _i32, _vp, _vp]),
    ("lc_plan_gemm_reserve", C.c_int, [_vp, _i32]),
    ("lc_plan_gemm_matrix", C.c_int, [_vp, C.POINTER(_vp)]),
    ("lc_autotune", C.c_int, [_vp, _vp]),
    ("lc_plan_destroy", C.c_int, [_vp]),
    ("lc_status_string", C.c_char_p, [C.c_int]),
    ("lc_last_error", C.c_char_p, []),
    ("lc_plan_set_timing", C.c_int, [_vp, _i32]),
    ("lc_plan_kernel_ms", C.c_int, [_vp, C.POINTER(C.c_double), _pi32]),
]

_lib = None


class LCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def load() -> C.CDLL:
    """Load ``liblc.so`` (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc, gfx950) first")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, what: str = "") -> None:
    if status != LC_OK:
        lib = load()
        msg = lib.lc_last_error().decode() or lib.lc_status_string(status).decode()
        if what and not msg.startswith(what):
            msg = f"{what}: {msg}"
        raise LCError(status, msg)
