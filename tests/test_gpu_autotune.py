"""The autotuner: choices keep the results (to rounding order) and persist
through the cache file named by LC_AUTOTUNE_CACHE."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import banner, expected_grid, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lc():
    import torch
    import paper_1106_0463_amd as lc
    torch.cuda.set_device(0)
    return lc


@pytest.mark.parametrize("N,M,Q", [(64, 256, 32), (3000, 12000, 48), (700, 82000, 12)])
def test_single_autotune_keeps_results(lc, tmp_path, N, M, Q):
    import torch
    banner(f"[gpu] autotune single N={N} M={M} Q={Q}")
    os.environ["LC_AUTOTUNE_CACHE"] = str(tmp_path / "cache.txt")
    f = W.Sum(W.Exponential(0.7), W.GeneratingFunction(0.6))
    p = lc.plan(N, M, Q)
    fx = f.torch(p.nodes).contiguous()
    c0 = p.execute(fx).clone()
    p.autotune()
    c1 = p.execute(fx).clone()
    torch.cuda.synchronize()
    ref = np.array(oracle.method_coeffs(f, N, expected_grid(M), Q), dtype=float)
    assert rel_err(c1.cpu().numpy(), ref) <= 1e-12
    assert rel_err(c1.cpu().numpy(), c0.cpu().numpy()) <= 1e-13
    # a second plan of the same shape takes the cached choice
    p2 = lc.plan(N, M, Q)
    p2.autotune()
    c2 = p2.execute(fx).clone()
    torch.cuda.synchronize()
    assert torch.equal(c1, c2)
    lines = open(tmp_path / "cache.txt").read().strip().splitlines()
    assert len(lines) == 1 and "|single|" in lines[0]
    p.destroy()
    p2.destroy()
    del os.environ["LC_AUTOTUNE_CACHE"]


def test_batch_autotune_keeps_results(lc):
    import torch
    from workloads.gpu import fill_closed_form_arena
    banner("[gpu] autotune batch")
    funcs = [W.GeneratingFunction(0.5), W.Exponential(-2.0), W.Cosine(20.0), W.GeneratingFunction(0.9)] * 8
    N = [64, 500, 1500, 9000] * 8
    M = [256, 2000, 6000, 36000] * 8
    Q = [32, 48, 48, 17] * 8
    prec = ["fp64", "fp32"] * 16
    bp = lc.plan_batch(N, M, Q, prec)
    f_off, x_off, c_off = bp.offsets()
    arena = torch.zeros(int(f_off[-1]) + 256, dtype=torch.uint8, device="cuda")
    H = [expected_grid(m) // 2 for m in M]
    fill_closed_form_arena(bp.nodes, arena, x_off, f_off, H, Q, funcs, [p == "fp32" for p in prec])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c0 = bp.execute(arena, stream=s).clone()
        bp.autotune(stream=s)
        c1 = bp.execute(arena, stream=s).clone()
        s.synchronize()
    # a new launch shape changes the FP64 summation order only
    for b in range(len(N)):
        a0 = c0[c_off[b]:c_off[b + 1]].cpu().numpy()
        a1 = c1[c_off[b]:c_off[b + 1]].cpu().numpy()
        assert rel_err(a1, a0) <= 1e-12, b
    bp.destroy()


def test_adaptive_autotune_keeps_results(lc, tmp_path):
    import torch
    banner("[gpu] autotune adaptive plan (lane groups)")
    os.environ["LC_AUTOTUNE_CACHE"] = str(tmp_path / "cache_a.txt")
    f = W.Sum(W.Cosine(900.0), W.GeneratingFunction(0.9))
    rule = dict(q=16, band=900.0, q_max=2048, grade_ratio=0.2, grade_levels=3)
    p = lc.plan_adaptive(1500, 6000, **rule)
    fx = f.torch(p.nodes).contiguous()
    c0 = p.execute(fx).clone()
    p.autotune()
    c1 = p.execute(fx).clone()
    torch.cuda.synchronize()
    assert rel_err(c1.cpu().numpy(), c0.cpu().numpy()) <= 5e-14
    with open(os.environ["LC_AUTOTUNE_CACHE"]) as fh:
        assert "adaptive" in fh.read()
    p.destroy()
    del os.environ["LC_AUTOTUNE_CACHE"]
