"""GPU checks of lc_execute_noalloc, the execute call of single plans whose
workspace is the library's static device array: its coefficients equal
those of lc_execute on the same plan and samples (same kernels, so bit for
bit), over calls in a row whose sizes shrink (the array keeps the previous
call's contents), for a four-step plan, an LDS-FFT plan, the one-kernel
small plan and a composite-rule plan; and a plan larger than the array is
rejected before any launch."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import banner, rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lc():
    import torch
    import paper_1106_0463_amd as lc
    torch.cuda.set_device(0)
    return lc


F = W.Sum(W.GeneratingFunction(0.6), W.Cosine(40.0))


def _both(lc, p, f):
    """(lc_execute result, lc_execute_noalloc result) on the same samples."""
    import torch
    fx = f.torch(p.nodes).contiguous()
    if p.info["precision"] == 1:
        fx = fx.float().contiguous()
    ref = p.execute(fx)
    out = torch.full((p.info["N"],), float("nan"), dtype=torch.float64, device="cuda")
    p.execute_noalloc(fx, out)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


# (N, M, Q): a four-step FFT (H = 131072: 3 MiB of workspace), then smaller
# LDS-FFT plans, then the one-kernel plan that needs no workspace at all
CALLS = [(20000, 262144, 8, "fp64"), (3000, 12000, 40, "fp64"), (700, 2400, 48, "fp32"),
         (64, 256, 32, "fp64")]


def test_noalloc_equals_execute_shrinking_calls(lc):
    for N, M, Q, prec in CALLS:
        banner(f"[gpu] lc_execute_noalloc vs lc_execute N={N} M={M} Q={Q} {prec}")
        p = lc.plan(N, M, Q, prec)
        ref, got = _both(lc, p, F)
        assert np.array_equal(ref, got), f"max diff {np.max(np.abs(ref - got)):.3e}"
        p.destroy()
    # the last LDS-FFT plan once more against the method oracle
    N, M, Q = 300, 1000, 24
    p = lc.plan(N, M, Q)
    ref, got = _both(lc, p, F)
    assert np.array_equal(ref, got)
    cm = np.array(oracle.method_coeffs(F, N, lc.grid_size(M), Q), dtype=float)
    assert rel_err(got, cm) <= 1e-12
    p.destroy()


def test_noalloc_adaptive_plan(lc):
    # a composite-rule plan with a breakpoint and graded panels, four-step
    # size first, then a smaller one
    for N, M in [(8000, 131072), (500, 2048)]:
        banner(f"[gpu] lc_execute_noalloc adaptive N={N} M={M}")
        p = lc.plan_adaptive(N, M, q=16, breaks=(0.25,), grade_ratio=0.25, grade_levels=3)
        ref, got = _both(lc, p, F)
        assert np.array_equal(ref, got), f"max diff {np.max(np.abs(ref - got)):.3e}"
        p.destroy()


def test_noalloc_rejects_plan_beyond_scratch(lc):
    import torch
    banner("[gpu] lc_execute_noalloc rejects H = 2^20")
    p = lc.plan(8, 1 << 21, 1)
    f = torch.zeros(p.info["samples"], dtype=torch.float64, device="cuda")
    out = torch.zeros(8, dtype=torch.float64, device="cuda")
    st = lc.load().lc_execute_noalloc(p._h, C.c_void_p(f.data_ptr()), C.c_void_p(out.data_ptr()), None)
    assert st == 1
    assert "static scratch" in lc.load().lc_last_error().decode()
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
    p.destroy()
