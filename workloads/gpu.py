"""GPU-side sampling of the synthetic inputs (torch for closed-form
families, the HIP Clenshaw sampler ``libsynth.so`` for random Legendre
series).  Input generation only."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsynth.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} not built (workloads.build.build())")
        lib = C.CDLL(LIB)
        vp = C.c_void_p
        lib.synth_series_ragged.argtypes = [C.c_int32, vp, vp, vp, vp, C.c_int64, vp, vp, vp, vp]
        lib.synth_series_ragged.restype = C.c_int
        lib.synth_series_grid.argtypes = [C.c_int32, C.c_int32, vp, C.c_int32, vp, vp, vp]
        lib.synth_series_grid.restype = C.c_int
        _lib = lib
    return _lib


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def series_ragged(coeffs, x_arena, x_off, f_arena, f_off, fp32):
    """Evaluate series b at nodes x_arena[x_off[b]:x_off[b+1]] into f_arena
    at byte offset f_off[b] (FP32 where fp32[b])."""
    import torch
    dev = x_arena.device
    B = len(coeffs)
    coef_off = np.zeros(B + 1, dtype=np.int64)
    coef_off[1:] = np.cumsum([len(c) for c in coeffs])
    coef = torch.from_numpy(np.concatenate(coeffs).astype(np.float64)).to(dev)
    t_coef_off = torch.from_numpy(coef_off).to(dev)
    t_x_off = torch.from_numpy(np.ascontiguousarray(x_off[:B + 1], dtype=np.int64)).to(dev)
    t_f_off = torch.from_numpy(np.ascontiguousarray(f_off[:B], dtype=np.int64)).to(dev)
    t_fp32 = torch.from_numpy(np.ascontiguousarray(fp32, dtype=np.int32)).to(dev)
    rc = _load().synth_series_ragged(B, C.c_void_p(coef.data_ptr()), C.c_void_p(t_coef_off.data_ptr()),
                                     C.c_void_p(x_arena.data_ptr()), C.c_void_p(t_x_off.data_ptr()),
                                     int(x_off[B]), C.c_void_p(f_arena.data_ptr()),
                                     C.c_void_p(t_f_off.data_ptr()), C.c_void_p(t_fp32.data_ptr()),
                                     _stream())
    if rc != 0:
        raise RuntimeError(f"synth_series_ragged failed ({rc})")
    torch.cuda.synchronize()


def series_grid(coef: np.ndarray, x_nodes, device="cuda"):
    """F[p][b] = sum_n coef[b][n] P_n(x_p), returned as a [P, B] float64 tensor."""
    import torch
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    B, ncoef = coef.shape
    tc = torch.from_numpy(coef).to(device)
    x = x_nodes.to(device=device, dtype=torch.float64).contiguous()
    P = x.numel()
    F = torch.empty((P, B), dtype=torch.float64, device=device)
    rc = _load().synth_series_grid(B, ncoef, C.c_void_p(tc.data_ptr()), P, C.c_void_p(x.data_ptr()),
                                   C.c_void_p(F.data_ptr()), _stream())
    if rc != 0:
        raise RuntimeError(f"synth_series_grid failed ({rc})")
    torch.cuda.synchronize()
    return F


def fill_closed_form_arena(nodes, f_arena, x_off, f_off, H, Q, funcs, fp32, omx=None):
    """Samples closed-form families f_b (objects with a .torch method) at
    their slices of the node arena into the byte arena (FP32 where fp32[b]).
    Given the arena of node complements 1 - x, families with a .torch_omx
    method are evaluated from it."""
    import torch
    for b, f in enumerate(funcs):
        n = int(H[b]) * int(Q[b])
        if omx is not None and hasattr(f, "torch_omx"):
            v = f.torch_omx(omx[int(x_off[b]):int(x_off[b]) + n])
        else:
            v = f.torch(nodes[int(x_off[b]):int(x_off[b]) + n])
        if fp32[b]:
            dst = f_arena[int(f_off[b]):int(f_off[b]) + 4 * n].view(torch.float32)
            dst.copy_(v.float())
        else:
            dst = f_arena[int(f_off[b]):int(f_off[b]) + 8 * n].view(torch.float64)
            dst.copy_(v)
    torch.cuda.synchronize()
