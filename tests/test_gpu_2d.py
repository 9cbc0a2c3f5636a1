"""GPU checks of two-dimensional tensor-product plans (the 1-D method along
x1 for every node of x2, then along x2): element-wise parity with the
oracle's 2-D transform on small and ragged sizes, closed-form separable
products at a larger size, and FP32 samples."""
import numpy as np
import pytest

import oracle
import workloads as W
from closed_forms import exp_coeffs
from helpers import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lc():
    import torch
    import paper_1106_0463_amd as lc
    torch.cuda.set_device(0)
    return lc


def _f2_np(x1, x2):
    return np.exp(x1 * x2) + x1 * x1 * np.cos(3 * x2)


def _f2_torch(x1, x2):
    import torch
    return torch.exp(x1 * x2) + x1 * x1 * torch.cos(3 * x2)


def _run(lc, N, M, Q, f2, precision="fp64"):
    import torch
    p = lc.plan_2d(N, M, Q, precision=precision)
    X = p.nodes.reshape(-1)
    F = f2(X[None, :], X[:, None]).contiguous()     # F[b][a] = f(X_a, X_b)
    if precision == "fp32":
        F = F.float().contiguous()
    C = p.execute(F)
    torch.cuda.synchronize()
    out = C.cpu().numpy()
    info = p.info
    p.destroy()
    return out, info


@pytest.mark.parametrize("N,M,Q", [(16, 64, 8), (33, 200, 7), (5, 12, 3)])
def test_2d_matches_oracle(lc, N, M, Q):
    from helpers import expected_grid
    banner(f"[gpu] 2-D plan vs oracle N={N} M={M} Q={Q}")
    got, info = _run(lc, N, M, Q, _f2_torch)
    Me = expected_grid(M)
    ref = np.asarray(oracle.method_coeffs_2d(_f2_np, N, Me, Q), dtype=float)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    banner(f"    rel err {err:.2e} (S = {info['H'] * info['Q']})")
    assert info["kind"] == 5 and info["samples"] == (info["H"] * info["Q"]) ** 2
    assert err <= 1e-13


def test_2d_separable_closed_forms(lc):
    import torch
    banner("[gpu] 2-D separable product vs closed forms N=128 M=512 Q=24")
    N, M, Q, t = 128, 512, 24, 0.4
    f2 = lambda x1, x2: torch.exp(0.9 * x1) * W.GeneratingFunction(t).torch(x2)
    got, _ = _run(lc, N, M, Q, f2)
    c1 = np.array([float(v) for v in exp_coeffs(0.9, N)])
    ref = np.outer(c1, t ** np.arange(N))
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    banner(f"    rel err {err:.2e}")
    assert err <= 1e-13


@pytest.mark.parametrize("N,M,Q,prec", [(16, 64, 8, "fp64"), (128, 512, 24, "fp64"), (64, 256, 16, "fp32"),
                                        (256, 1024, 32, "fp64")])
def test_2d_row_pairs(lc, monkeypatch, N, M, Q, prec):
    # both passes' reductions over row pairs (LC_2D_ROW_PAIRS=1) against the
    # one-row shapes (another summation order) and, for FP64 samples, the
    # 2-D method oracle
    from helpers import expected_grid
    banner(f"[gpu] 2-D row pairs N={N} M={M} Q={Q} {prec}")
    monkeypatch.setenv("LC_2D_ROW_PAIRS", "0")
    c1, _ = _run(lc, N, M, Q, _f2_torch, precision=prec)
    monkeypatch.setenv("LC_2D_ROW_PAIRS", "1")
    c2, _ = _run(lc, N, M, Q, _f2_torch, precision=prec)
    d = np.max(np.abs(c2 - c1)) / np.max(np.abs(c1))
    banner(f"    difference to one row per lane group {d:.2e}")
    assert d <= 1e-13
    if prec == "fp64" and N <= 16:
        ref = np.asarray(oracle.method_coeffs_2d(_f2_np, N, expected_grid(M), Q), dtype=float)
        assert np.max(np.abs(c2 - ref)) / np.max(np.abs(ref)) <= 1e-13


def test_2d_fp32_samples(lc):
    banner("[gpu] 2-D FP32 samples vs FP64")
    N, M, Q = 64, 256, 16
    c64, _ = _run(lc, N, M, Q, _f2_torch)
    c32, _ = _run(lc, N, M, Q, _f2_torch, precision="fp32")
    n = np.arange(N)
    scale = np.outer(2 * n + 1, 2 * n + 1)
    E_a = np.max(np.abs((c32 - c64) / scale)) / np.max(np.abs(c64 / scale))
    banner(f"    E_a {E_a:.2e}")
    assert E_a <= 1e-7


def test_2d_bench_size(lc):
    # the benchmark's size N = 256, M = 1024, Q = 32 (S = 16384 nodes per
    # axis, 2.7e8 samples), element by element:
    #  * a rank-two separable f: the method is linear and acts on each axis
    #    alone, so its 2-D result is the sum of outer products of the 1-D
    #    method oracle's coefficients at the same (N, M, Q);
    #  * the benchmark's f = exp(x1 x2) + x1^2 cos(3 x2) against eq. (2.3)
    #    along both axes (a 304-point long-double Gauss-Legendre rule per axis)
    import torch
    from helpers import expected_grid
    N, M, Q = 256, 1024, 32
    Me = expected_grid(M)
    banner(f"[gpu] 2-D plan at the benchmark size N={N} M={M} Q={Q}")
    g1, h1 = W.Exponential(0.9), W.GeneratingFunction(0.4)
    g2, h2 = W.Cosine(3.0), W.Exponential(-1.7)
    f2 = lambda x1, x2: g1.torch(x1) * h1.torch(x2) + g2.torch(x1) * h2.torch(x2)
    got, info = _run(lc, N, M, Q, f2)
    assert info["H"] * info["Q"] == 16384
    cm = {k: np.array(oracle.method_coeffs(f, N, Me, Q, fp64_nodes=True), dtype=float)
          for k, f in (("g1", g1), ("h1", h1), ("g2", g2), ("h2", h2))}
    ref = np.outer(cm["g1"], cm["h1"]) + np.outer(cm["g2"], cm["h2"])
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    banner(f"    separable: rel err {err:.2e} vs the 1-D method oracle")
    assert err <= 1e-13
    got, _ = _run(lc, N, M, Q, _f2_torch)
    K = N + 48
    x, w = oracle.gauss_legendre(K)
    xl = x.astype(np.longdouble)
    Fk = np.exp(xl[:, None] * xl[None, :]) + xl[:, None] ** 2 * np.cos(3 * xl[None, :])  # [k1][k2]
    step1 = np.stack([oracle.legendre_coeffs_from_samples(x, w, Fk[:, k], N) for k in range(K)], axis=1)
    ref = np.stack([oracle.legendre_coeffs_from_samples(x, w, step1[n, :], N) for n in range(N)], axis=0)
    ref = np.asarray(ref, dtype=float)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    banner(f"    exp(x1 x2) + x1^2 cos(3 x2): rel err {err:.2e} vs eq. (2.3) along both axes")
    assert err <= 1e-12
