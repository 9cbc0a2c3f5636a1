"""Fixed-grid plans: functions sampled on one Chebyshev-Gauss grid
(binding of lc_plan_gemm, lc_plan_legendre_matrix and lc_execute_gemm)."""
from __future__ import annotations

import ctypes as C

from . import Plan, _check_out, _stream_handle, _view
from ._lib import GEMM_MODES, check, load


class GemmPlan(Plan):
    @property
    def matrix(self):
        """FP64 matrix of the plan (device view): the product-integration
        matrix A [H+1, P], or Lmat^T [P, N] for a Legendre-matrix plan."""
        ptr = C.c_void_p()
        check(self._lib.lc_plan_gemm_matrix(self._h, C.byref(ptr)), "lc_plan_gemm_matrix")
        info = self.info
        if info["kind"] == LEGENDRE_MATRIX:
            return _view(ptr.value, (info["Q"], info["N"]), self)
        return _view(ptr.value, (info["H"] + 1, info["Q"]), self)

    def reserve(self, B: int) -> None:
        check(self._lib.lc_plan_gemm_reserve(self._h, int(B)), "lc_plan_gemm_reserve")
        self._info = None

    def execute(self, F, out=None, stream=None):
        """F: float64 CUDA tensor [P, B]; returns C [B, N] (float64)."""
        import torch
        info = self.info
        P, N = info["Q"], info["N"]
        if F.dtype != torch.float64 or not F.is_cuda or not F.is_contiguous() or F.dim() != 2 \
                or F.shape[0] != P:
            raise ValueError(f"F must be a contiguous float64 CUDA tensor [{P}, B]")
        B = F.shape[1]
        if out is None:
            out = torch.empty((B, N), dtype=torch.float64, device=F.device)
        else:
            _check_out(out, B * N, "out", F.device)
        check(self._lib.lc_execute_gemm(self._h, C.c_void_p(F.data_ptr()), int(B),
                                        C.c_void_p(out.data_ptr()), _stream_handle(stream)),
              "lc_execute_gemm")
        return out


LEGENDRE_MATRIX = 3  # lc_plan_kind of lc_plan_legendre_matrix plans


def plan_gemm(P: int, M: int, N: int, mode: str = "fp16x3") -> GemmPlan:
    """Abel product phi = A F, then the batched twist/FFT/rescale.  The
    default fp16x3 and bf16x6 hold E_a <= 1e-7 (the mixed class); bf16x3
    and fp16x1 are faster and less accurate (outside that class)."""
    h = C.c_void_p()
    check(load().lc_plan_gemm(int(P), int(M), int(N), GEMM_MODES[mode], C.byref(h)), "lc_plan_gemm")
    return GemmPlan(h)


def plan_legendre_matrix(P: int, M: int, N: int, mode: str = "fp16x3") -> GemmPlan:
    """One product C = F^T Lmat^T with the FP64-built N x P Legendre matrix
    (modes and classes as in :func:`plan_gemm`)."""
    h = C.c_void_p()
    check(load().lc_plan_legendre_matrix(int(P), int(M), int(N), GEMM_MODES[mode], C.byref(h)),
          "lc_plan_legendre_matrix")
    return GemmPlan(h)
