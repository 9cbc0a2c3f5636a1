"""MI355X-native Legendre coefficients by the Abel-transform + FFT method of
De Micheli & Viano (arXiv 1106.0463).

Thin Python binding over the C ABI of ``include/lc.h``.  torch is used for
device memory and streams only; every step of the method runs in the HIP
library ``liblc.so`` (built for gfx950).  There is no CPU fallback: without
the library, or without a GPU, calls raise.

Typical use::

    import torch, paper_1106_0463_amd as lc
    p = lc.plan(N=64, M=256, Q=32)          # nodes x[H][Q] on the GPU
    f = my_function(p.nodes)                # sample f at the nodes (torch)
    c = p.execute(f)                        # c_0..c_{N-1}, float64 tensor
"""
from __future__ import annotations

import ctypes as C

from ._lib import (GEMM_MODES, LC_FP32_QUAD, LC_FP64, PRECISIONS, LCError,  # noqa: F401
                   PlanDesc, check, load)

__all__ = ["grid_size", "plan", "plan_2d", "plan_adaptive", "plan_batch", "plan_batch_rules", "plan_gemm", "plan_legendre_matrix",
           "Plan", "Plan2D", "LCError"]


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _check_out(out, n: int, what: str, device=None) -> None:
    """A caller-supplied output buffer must be a contiguous float64 CUDA
    tensor of at least n elements (the kernels write n doubles into it),
    on the device of the inputs when one is given."""
    torch = _torch()
    if (not isinstance(out, torch.Tensor) or out.dtype != torch.float64 or not out.is_cuda
            or not out.is_contiguous() or out.numel() < int(n)):
        raise ValueError(f"{what} must be a contiguous float64 CUDA tensor of at least {int(n)} elements")
    if device is not None and out.device != device:
        raise ValueError(f"{what} must be on {device}")


def grid_size(M: int) -> int:
    """Effective y-grid size the library uses for a requested M."""
    out = C.c_int64()
    check(load().lc_grid_size(int(M), C.byref(out)), "lc_grid_size")
    return int(out.value)


class _DevArray:
    """Zero-copy view of library-owned device memory for torch."""

    def __init__(self, ptr: int, shape, typestr: str, owner):
        self._owner = owner
        self.__cuda_array_interface__ = {
            "shape": tuple(int(s) for s in shape), "typestr": typestr,
            "data": (int(ptr), False), "version": 2, "strides": None}


def _view(ptr: int, shape, owner, dtype="float64"):
    torch = _torch()
    typestr = {"float64": "<f8"}[dtype]
    t = torch.as_tensor(_DevArray(ptr, shape, typestr, owner), device="cuda")
    return t


class Plan:
    """A plan created by :func:`plan`, :func:`plan_batch` or :func:`plan_gemm`."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle
        self._lib = load()
        self._info = None

    # -- lifetime -----------------------------------------------------
    def destroy(self) -> None:
        if self._h:
            self._lib.lc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.destroy()

    # -- description --------------------------------------------------
    @property
    def info(self) -> dict:
        """Plan description (lc_plan_info), cached: single and batch plans
        never change shape; GEMM plans refresh it on reserve."""
        if self._info is None:
            d = PlanDesc()
            check(self._lib.lc_plan_info(self._h, C.byref(d)), "lc_plan_info")
            self._info = {k: getattr(d, k) for k, _ in PlanDesc._fields_}
        return self._info

    @property
    def nodes(self):
        """Device nodes (float64 tensor view owned by the plan): [H, Q] for a
        single plan, the flat node arena for a batch plan, [P] for GEMM."""
        ptr, rows, q = C.c_void_p(), C.c_int64(), C.c_int32()
        check(self._lib.lc_plan_nodes(self._h, C.byref(ptr), C.byref(rows), C.byref(q)),
              "lc_plan_nodes")
        info = self.info
        if info["kind"] in (0, 5):  # single and 2-D plans: [H, Q]
            return _view(ptr.value, (rows.value, q.value), self)
        return _view(ptr.value, (rows.value,), self)

    def nodes_complement(self, stream=None):
        """1 - x for every node (lc_plan_nodes_complement), a float64 CUDA
        tensor shaped like :attr:`nodes` (single, adaptive and batch plans)."""
        torch = _torch()
        x = self.nodes
        out = torch.empty_like(x)
        check(self._lib.lc_plan_nodes_complement(self._h, C.c_void_p(out.data_ptr()), _stream_handle(stream)),
              "lc_plan_nodes_complement")
        return out

    # -- execution ----------------------------------------------------
    def execute(self, f, out=None, stream=None):
        """c_0..c_{N-1} from samples f[H][Q] (float64, or float32 for an
        'fp32' plan) on the GPU; asynchronous on ``stream``."""
        torch = _torch()
        info = self.info
        want = torch.float64 if info["precision"] == LC_FP64 else torch.float32
        if f.dtype != want or not f.is_cuda or not f.is_contiguous():
            raise ValueError(f"f must be a contiguous {want} CUDA tensor")
        if f.numel() != info["samples"]:
            raise ValueError(f"f has {f.numel()} samples, plan expects {info['samples']}")
        if out is None:
            out = torch.empty(info["N"], dtype=torch.float64, device=f.device)
        else:
            _check_out(out, info["N"], "out", f.device)
        check(self._lib.lc_execute(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()),
                                   _stream_handle(stream)), "lc_execute")
        return out

    def execute_noalloc(self, f, out, stream=None):
        """lc_execute_noalloc: as ``execute`` with the workspace in the
        library's static device array; ``out`` (N float64 values) is
        required, so that nothing is allocated."""
        torch = _torch()
        info = self.info
        want = torch.float64 if info["precision"] == LC_FP64 else torch.float32
        if f.dtype != want or not f.is_cuda or not f.is_contiguous():
            raise ValueError(f"f must be a contiguous {want} CUDA tensor")
        if f.numel() != info["samples"]:
            raise ValueError(f"f has {f.numel()} samples, plan expects {info['samples']}")
        _check_out(out, info["N"], "out", f.device)
        check(self._lib.lc_execute_noalloc(self._h, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()),
                                           _stream_handle(stream)), "lc_execute_noalloc")
        return out

    def set_timing(self, enable: bool = True) -> None:
        check(self._lib.lc_plan_set_timing(self._h, 1 if enable else 0), "lc_plan_set_timing")

    def kernel_ms(self) -> tuple[float, int]:
        ms, n = C.c_double(), C.c_int32()
        check(self._lib.lc_plan_kernel_ms(self._h, C.byref(ms), C.byref(n)), "lc_plan_kernel_ms")
        return float(ms.value), int(n.value)

    def autotune(self, stream=None) -> None:
        check(self._lib.lc_autotune(self._h, _stream_handle(stream)), "lc_autotune")


def plan(N: int, M: int, Q: int, precision: str = "fp64") -> Plan:
    """Single-function plan: N coefficients, M-point y-grid, Q Abel nodes."""
    h = C.c_void_p()
    check(load().lc_plan(int(N), int(M), int(Q), PRECISIONS[precision], C.byref(h)), "lc_plan")
    return Plan(h)


def plan_adaptive(N: int, M: int, q: int, band: float = 0.0, q_max: int = 0, breaks=(),
                  grade_ratio: float = 0.0, grade_levels: int = 0, precision: str = "fp64") -> Plan:
    """Single-function plan with the composite Abel rule (lc_abel_rule):
    breakpoints of f, geometric grading toward x = 1 and per-row node
    counts for f band-limited to degree ``band``.  Nodes and samples are one
    flat array (``Plan.nodes``)."""
    from ._lib import AbelRule
    br = (C.c_double * max(1, len(breaks)))(*[float(b) for b in breaks])
    rule = AbelRule(int(q), int(q_max), float(band), len(breaks), br, float(grade_ratio), int(grade_levels))
    h = C.c_void_p()
    check(load().lc_plan_adaptive(int(N), int(M), C.byref(rule), PRECISIONS[precision], C.byref(h)),
          "lc_plan_adaptive")
    return Plan(h)


class Plan2D(Plan):
    """Two-dimensional tensor-product plan (lc_plan_2d): both axes use the
    S = H Q nodes of ``nodes`` (flattened); samples F[b, a] = f(X_a, X_b)."""

    def execute(self, F, out=None, stream=None):
        """C[n1, n2] (float64 N x N) from the S x S samples F on the GPU."""
        torch = _torch()
        info = self.info
        want = torch.float64 if info["precision"] == LC_FP64 else torch.float32
        S = info["H"] * info["Q"]
        if F.dtype != want or not F.is_cuda or not F.is_contiguous() or F.numel() != S * S:
            raise ValueError(f"F must be a contiguous {want} CUDA tensor of {S} x {S} samples")
        N = info["N"]
        if out is None:
            out = torch.empty((N, N), dtype=torch.float64, device=F.device)
        else:
            _check_out(out, N * N, "out", F.device)
        check(self._lib.lc_execute_2d(self._h, C.c_void_p(F.data_ptr()), C.c_void_p(out.data_ptr()),
                                      _stream_handle(stream)), "lc_execute_2d")
        return out


def plan_2d(N: int, M: int, Q: int, precision: str = "fp64") -> Plan2D:
    """Two-dimensional plan: N x N coefficients, the 1-D grid (M, Q) on both axes."""
    h = C.c_void_p()
    check(load().lc_plan_2d(int(N), int(M), int(Q), PRECISIONS[precision], C.byref(h)), "lc_plan_2d")
    return Plan2D(h)


from .batch import BatchPlan, plan_batch, plan_batch_rules, rule_row_length  # noqa: E402,F401
from .gemm import GemmPlan, plan_gemm, plan_legendre_matrix  # noqa: E402,F401
