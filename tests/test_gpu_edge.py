"""Edge cases and determinism across plan kinds: repeated executes are
bitwise identical; degenerate sizes (N = 1, the smallest grids, one Abel
node, one function, P = 2) against the oracle or the method's exactness;
an adaptive rule with many breakpoints against the oracle's rule."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

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


def _twice(fn):
    import torch
    a = fn().clone()
    b = fn().clone()
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_determinism_every_plan_kind(lc):
    import torch
    from workloads.gpu import series_grid
    banner("[gpu] repeated executes are bitwise identical")
    f = W.Sum(W.Exponential(0.7), W.GeneratingFunction(0.6))
    p = lc.plan(300, 1200, 24)
    fx = f.torch(p.nodes).contiguous()
    a, b = _twice(lambda: p.execute(fx))
    assert np.array_equal(a, b)
    pa = lc.plan_adaptive(300, 1200, q=16, breaks=(0.3,), grade_ratio=0.2, grade_levels=3)
    fa = f.torch(pa.nodes).contiguous()
    a, b = _twice(lambda: pa.execute(fa))
    assert np.array_equal(a, b)
    p2 = lc.plan_2d(16, 64, 8)
    X = p2.nodes.reshape(-1)
    F2 = torch.exp(X[None, :] * X[:, None]).contiguous()
    a, b = _twice(lambda: p2.execute(F2))
    assert np.array_equal(a, b)
    coef = W.gemm_batch_coeffs(40, 200, seed=11)
    for mk in (lambda: lc.plan_gemm(256, 512, 200, "fp16x3"), lambda: lc.plan_legendre_matrix(256, 512, 200, "bf16x6")):
        g = mk()
        F = series_grid(coef, g.nodes)
        a, b = _twice(lambda: g.execute(F))
        assert np.array_equal(a, b)
        g.destroy()
    for q in (p, pa, p2):
        q.destroy()


@pytest.mark.parametrize("N,M,q", [(1, 4, 1), (1, 2, 3), (2, 8, 2)])
def test_smallest_single_and_adaptive(lc, N, M, q):
    banner(f"[gpu] smallest plans N={N} M={M} q={q}")
    f = W.Exponential(0.5)
    Me = expected_grid(M)
    ref = np.array(oracle.method_coeffs(f, N, Me, q, fp64_nodes=True), dtype=float)
    p = lc.plan(N, M, q)
    c = p.execute(f.torch(p.nodes).contiguous()).cpu().numpy()
    p.destroy()
    pa = lc.plan_adaptive(N, M, q=q)
    ca = pa.execute(f.torch(pa.nodes).contiguous()).cpu().numpy()
    pa.destroy()
    assert rel_err(c, ref) <= 1e-14
    assert rel_err(ca, ref) <= 1e-14


def test_many_breakpoints_against_oracle(lc):
    banner("[gpu] adaptive rule with 64 breakpoints vs the oracle's rule")
    brk = tuple(np.linspace(-0.95, 0.95, 64))
    rule = dict(q=8, breaks=brk)
    f = W.AbsPower(1.5)
    N, M = 48, 256
    p = lc.plan_adaptive(N, M, **rule)
    c = p.execute(f.torch(p.nodes).contiguous()).cpu().numpy()
    p.destroy()
    ref = np.array(oracle.method_coeffs_rule(f, N, expected_grid(M), dict(rule), fp64_nodes=True), dtype=float)
    assert rel_err(c, ref) <= 1e-13


def test_2d_single_coefficient(lc):
    import torch
    banner("[gpu] 2-D plan with N = 1")
    p = lc.plan_2d(1, 8, 4)
    X = p.nodes.reshape(-1)
    F = (2.0 + X[None, :] * X[:, None]).contiguous()
    c = p.execute(F).cpu().numpy()
    p.destroy()
    # c_00 = (1/4) integral integral (2 + x1 x2) = 2
    assert abs(c[0, 0] - 2.0) <= 1e-14


@pytest.mark.parametrize("kind", ["gemm", "matrix"])
def test_fixed_grid_tiny(lc, kind):
    from workloads.gpu import series_grid
    banner(f"[gpu] {kind}: P = 2, one function; P = 33 ragged")
    mk = lc.plan_gemm if kind == "gemm" else lc.plan_legendre_matrix
    # P = 2 nodes, degree 1, M = 4: exact
    coef = np.array([[0.5, -1.25]])
    g = mk(2, 4, 2, "fp64")
    C = g.execute(series_grid(coef, g.nodes)).cpu().numpy()
    g.destroy()
    assert np.max(np.abs(C - coef)) <= 1e-14
    coef = W.gemm_batch_coeffs(3, 20, seed=12)
    g = mk(33, 128, 40, "fp16x3")
    C = g.execute(series_grid(coef, g.nodes)).cpu().numpy()
    g.destroy()
    ref = np.zeros((3, 40))
    ref[:, :21] = coef
    n = np.arange(40)
    assert rel_err(C / (2 * n + 1), ref / (2 * n + 1)) <= 1e-7


def test_output_buffers_validated_before_launch(lc):
    # a wrong dtype, a short buffer, a strided view or a host tensor as the
    # output of any execute raises ValueError before anything is launched;
    # the buffer is left untouched
    import torch
    banner("[gpu] output buffers: dtype, size, contiguity and device checked")
    f = W.Exponential(0.5)
    p = lc.plan(20, 64, 8)
    fx = f.torch(p.nodes).contiguous()
    bad = [torch.zeros(20, dtype=torch.float32, device="cuda"),
           torch.zeros(19, dtype=torch.float64, device="cuda"),
           torch.zeros(40, dtype=torch.float64, device="cuda")[::2],
           torch.zeros(20, dtype=torch.float64)]
    for out in bad:
        with pytest.raises(ValueError):
            p.execute(fx, out)
    p.destroy()
    p2 = lc.plan_2d(4, 16, 3)
    X = p2.nodes.reshape(-1)
    F2 = torch.exp(X[None, :] * X[:, None]).contiguous()
    for out in (torch.zeros(15, dtype=torch.float64, device="cuda"),
                torch.zeros(16, dtype=torch.float32, device="cuda")):
        with pytest.raises(ValueError):
            p2.execute(F2, out)
        assert int(torch.count_nonzero(out)) == 0
    p2.destroy()
    bp = lc.plan_batch([5, 9], [16, 40], [4, 6], "fp64")
    f_off, _, c_off = bp.offsets()
    arena = torch.zeros(int(f_off[-1]), dtype=torch.uint8, device="cuda")
    for out in (torch.zeros(int(c_off[-1]) - 1, dtype=torch.float64, device="cuda"),
                torch.zeros(int(c_off[-1]), dtype=torch.float32, device="cuda")):
        with pytest.raises(ValueError):
            bp.execute(arena, out)
        assert int(torch.count_nonzero(out)) == 0
    with pytest.raises(ValueError):
        bp.execute(arena[: int(f_off[-1]) - 8])
    bp.destroy()
    from workloads.gpu import series_grid
    g = lc.plan_gemm(32, 64, 16, "fp16x3")
    F = series_grid(W.gemm_batch_coeffs(3, 10, seed=13), g.nodes)
    for out in (torch.zeros((3, 15), dtype=torch.float64, device="cuda"),
                torch.zeros((3, 16), dtype=torch.float32, device="cuda")):
        with pytest.raises(ValueError):
            g.execute(F, out)
        assert int(torch.count_nonzero(out)) == 0
    g.destroy()


def test_out_of_memory_status():
    """LC_ERR_NOMEM through the LC_ALLOC_LIMIT hook (any device allocation
    above the limit fails), in a child process so that the limit holds from
    the library's first allocation: every plan kind reports LC_ERR_NOMEM,
    leaves *out untouched and says what failed; a plan below the limit still
    builds and runs."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = r'''
import ctypes as C, sys
sys.path.insert(0, %r)
import paper_1106_0463_amd as lc
from paper_1106_0463_amd._lib import AbelRule
lib = lc.load()
def check(st, h, what):
    assert st == 2 and h.value == 777, (what, st, h.value, lib.lc_last_error())
    assert lib.lc_last_error().decode() != "", what
h = C.c_void_p(777)
check(lib.lc_plan(1000, 4000, 48, 0, C.byref(h)), h, "lc_plan")
rule = AbelRule(16, 0, 0.0, 0, None, 0.2, 3)
check(lib.lc_plan_adaptive(1000, 4000, C.byref(rule), 0, C.byref(h)), h, "lc_plan_adaptive")
N = (C.c_int64 * 2)(500, 40); M = (C.c_int64 * 2)(2000, 160); Q = (C.c_int32 * 2)(48, 48); P = (C.c_int * 2)(0, 1)
check(lib.lc_plan_batch(2, N, M, Q, P, C.byref(h)), h, "lc_plan_batch")
check(lib.lc_plan_gemm(512, 2048, 1000, 3, C.byref(h)), h, "lc_plan_gemm")
assert lib.lc_plan(8, 16, 2, 0, C.byref(h)) == 0
assert lib.lc_plan_destroy(h) == 0
print("NOMEM_OK")
''' % root
    env = dict(os.environ, LC_ALLOC_LIMIT="65536")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "NOMEM_OK" in r.stdout, r.stdout + r.stderr


def test_plan_log():
    """LC_LOG=1 prints one line per plan decision on stderr (grid size, launch
    shapes, radix schedules, batch classes and DST groups); without it the
    library prints nothing."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = r'''
import sys
sys.path.insert(0, %r)
import paper_1106_0463_amd as lc
lc.plan(100, 300, 17).destroy()
lc.plan(700, 82000, 12).destroy()
lc.plan(1000, 8192, 48).destroy()
lc.plan_adaptive(64, 512, q=16, grade_ratio=0.2, grade_levels=3).destroy()
lc.plan_batch([30, 300], [120, 1200], [48, 24], ["fp64", "fp32"]).destroy()
lc.plan_gemm(64, 256, 100, "fp16x3").destroy()
''' % root
    for log in ("1", "0"):
        env = dict(os.environ, LC_LOG=log)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        lines = [s for s in r.stderr.splitlines() if s.startswith("[lc]")]
        if log == "0":
            assert not lines, lines
            continue
        text = "\n".join(lines)
        for want in ("lc_plan: N=100 M=300 M_eff=", "one fused kernel", "four-step", "LDS FFT L=2048", "lc_plan_adaptive: N=64",
                     "lc_plan_batch: B=2", "class R=48 fp64", "class R=24 fp32", "DST group", "lc_plan_gemm: P=64"):
            assert want in text, (want, text)
