"""Batched plans: many functions of uneven N/M/Q in one graph-captured
execution (binding of lc_plan_batch / lc_execute_batch)."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import Plan, _check_out, _stream_handle, _view
from ._lib import PRECISIONS, check, load


class BatchPlan(Plan):
    def offsets(self):
        """(f_off bytes, x_off elements, c_off elements), each of length B+1."""
        if getattr(self, "_offsets", None) is not None:
            return self._offsets
        B = self.info["B"]
        f = np.zeros(B + 1, dtype=np.int64)
        x = np.zeros(B + 1, dtype=np.int64)
        c = np.zeros(B + 1, dtype=np.int64)
        p = lambda a: a.ctypes.data_as(C.POINTER(C.c_int64))
        check(self._lib.lc_plan_batch_offsets(self._h, p(f), p(x), p(c)), "lc_plan_batch_offsets")
        self._offsets = (f, x, c)
        return self._offsets

    @property
    def nodes(self):
        ptr, rows, q = C.c_void_p(), C.c_int64(), C.c_int32()
        check(self._lib.lc_plan_nodes(self._h, C.byref(ptr), C.byref(rows), C.byref(q)),
              "lc_plan_nodes")
        return _view(ptr.value, (rows.value,), self)

    def execute(self, f_arena, c_arena=None, stream=None):
        """f_arena: uint8 (or any dtype) CUDA tensor holding the sample arena
        (layout of :meth:`offsets`); returns the float64 coefficient arena."""
        import torch
        f_off, _, c_off = self.offsets()
        if (not isinstance(f_arena, torch.Tensor) or not f_arena.is_cuda or not f_arena.is_contiguous()
                or f_arena.numel() * f_arena.element_size() < f_off[-1]):
            raise ValueError(f"f_arena must be a contiguous CUDA tensor of at least {int(f_off[-1])} bytes")
        if c_arena is None:
            c_arena = torch.empty(int(c_off[-1]), dtype=torch.float64, device=f_arena.device)
        else:
            _check_out(c_arena, int(c_off[-1]), "c_arena", f_arena.device)
        check(self._lib.lc_execute_batch(self._h, C.c_void_p(f_arena.data_ptr()),
                                         C.c_void_p(c_arena.data_ptr()), _stream_handle(stream)),
              "lc_execute_batch")
        return c_arena


def plan_batch(N, M, Q, precision) -> BatchPlan:
    """N, M, Q: integer sequences of length B; precision: sequence of
    'fp64' / 'fp32' (or one string for all)."""
    N = np.ascontiguousarray(N, dtype=np.int64)
    M = np.ascontiguousarray(M, dtype=np.int64)
    Q = np.ascontiguousarray(Q, dtype=np.int32)
    B = N.size
    if isinstance(precision, str):
        precision = [precision] * B
    pr = np.ascontiguousarray([PRECISIONS[p] for p in precision], dtype=np.int32)
    if not (M.size == Q.size == pr.size == B):
        raise ValueError("N, M, Q, precision must have one length")
    h = C.c_void_p()
    check(load().lc_plan_batch(int(B), N.ctypes.data_as(C.POINTER(C.c_int64)),
                               M.ctypes.data_as(C.POINTER(C.c_int64)),
                               Q.ctypes.data_as(C.POINTER(C.c_int32)),
                               pr.ctypes.data_as(C.POINTER(C.c_int)), C.byref(h)), "lc_plan_batch")
    return BatchPlan(h)


def rule_row_length(rule: dict) -> int:
    """Samples per row R of a batch rule (lc_plan_batch_rules):
    (grade_levels + 1) * (q rounded up to a multiple of 4)."""
    q = int(rule["q"])
    levels = int(rule.get("grade_levels", 0)) if float(rule.get("grade_ratio", 0.0)) > 0 else 0
    return (levels + 1) * ((q + 3) // 4 * 4)


def plan_batch_rules(N, M, rules, precision) -> BatchPlan:
    """N, M: integer sequences of length B; rules: sequence of dicts with
    keys q, grade_ratio, grade_levels (lc_abel_rule without band or
    breakpoints); precision: sequence of 'fp64' / 'fp32' (or one string)."""
    from ._lib import AbelRule
    N = np.ascontiguousarray(N, dtype=np.int64)
    M = np.ascontiguousarray(M, dtype=np.int64)
    B = N.size
    if isinstance(precision, str):
        precision = [precision] * B
    pr = np.ascontiguousarray([PRECISIONS[p] for p in precision], dtype=np.int32)
    if not (M.size == len(rules) == pr.size == B):
        raise ValueError("N, M, rules, precision must have one length")
    arr = (AbelRule * B)()
    for b, r in enumerate(rules):
        arr[b] = AbelRule(int(r["q"]), int(r.get("q_max", 0)), float(r.get("band", 0.0)), 0, None,
                          float(r.get("grade_ratio", 0.0)), int(r.get("grade_levels", 0)))
    h = C.c_void_p()
    check(load().lc_plan_batch_rules(int(B), N.ctypes.data_as(C.POINTER(C.c_int64)),
                                     M.ctypes.data_as(C.POINTER(C.c_int64)), arr,
                                     pr.ctypes.data_as(C.POINTER(C.c_int)), C.byref(h)), "lc_plan_batch_rules")
    return BatchPlan(h)
