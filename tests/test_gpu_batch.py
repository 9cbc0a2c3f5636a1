"""GPU parity of the batched path (ragged batches in one graph launch)
against the CPU oracle, the single-function path and the exact
coefficients of random finite Legendre series."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from helpers import banner, expected_grid, rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def lc():
    import torch
    import paper_1106_0463_amd as lc
    torch.cuda.set_device(0)
    return lc


def _build(lc, funcs, N, M, Q, prec):
    import torch
    from workloads.gpu import fill_closed_form_arena
    bp = lc.plan_batch(N, M, Q, prec)
    f_off, x_off, c_off = bp.offsets()
    nodes = bp.nodes
    H = [expected_grid(m) // 2 for m in M]
    arena = torch.zeros(int(f_off[-1]) + 256, dtype=torch.uint8, device="cuda")
    fill_closed_form_arena(nodes, arena, x_off, f_off, H, Q, funcs, [p == "fp32" for p in prec])
    return bp, arena, c_off


SMALL = [  # (family, N, M, Q, precision)
    (W.GeneratingFunction(0.5), 64, 256, 32, "fp64"),
    (W.Exponential(1.0), 64, 256, 32, "fp64"),
    (W.Exponential(-3.0), 700, 2000, 48, "fp64"),
    (W.GeneratingFunction(0.8), 1, 2, 1, "fp64"),
    (W.Cosine(40.0), 3000, 12000, 48, "fp32"),
    (W.Sum(W.Exponential(0.7), W.GeneratingFunction(0.6)), 5000, 40000, 33, "fp64"),
    (W.Rational(2.0), 333, 1000, 7, "fp32"),
    (W.GeneratingFunction(0.3), 4096, 8192, 64, "fp64"),
    (W.Exponential(5.0), 100, 300, 16, "fp32"),
    (W.Cosine(10.0), 129, 600, 48, "fp64"),
    (W.GeneratingFunction(0.9), 9000, 36000, 48, "fp64"),
    (W.Exponential(-1.0), 2, 4, 3, "fp64"),
]


def test_small_ragged_batch(lc):
    import torch
    banner(f"[gpu] ragged batch of {len(SMALL)}")
    funcs = [s[0] for s in SMALL]
    N = [s[1] for s in SMALL]
    M = [s[2] for s in SMALL]
    Q = [s[3] for s in SMALL]
    prec = [s[4] for s in SMALL]
    bp, arena, c_off = _build(lc, funcs, N, M, Q, prec)
    c = bp.execute(arena)
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    for b, (f, n, m, q, pr) in enumerate(SMALL):
        got = c[c_off[b]:c_off[b + 1]]
        ref = np.array(oracle.method_coeffs(f, n, expected_grid(m), q), dtype=float)
        if pr == "fp64":
            assert rel_err(got, ref) <= TOL, b
        else:
            k = 2 * np.arange(n) + 1
            assert rel_err(got / k, ref / k) <= 1e-7, b
    bp.destroy()


def test_batch_matches_single_plans(lc):
    import torch
    banner("[gpu] batch vs single plans")
    funcs = [s[0] for s in SMALL]
    N = [s[1] for s in SMALL]
    M = [s[2] for s in SMALL]
    Q = [s[3] for s in SMALL]
    prec = [s[4] for s in SMALL]
    bp, arena, c_off = _build(lc, funcs, N, M, Q, prec)
    c = bp.execute(arena).cpu().numpy()
    for b, (f, n, m, q, pr) in enumerate(SMALL):
        p = lc.plan(n, m, q, pr)
        fx = f.torch(p.nodes).contiguous()
        if pr == "fp32":
            fx = fx.float().contiguous()
        cs = p.execute(fx)
        torch.cuda.synchronize()
        # different reduction orders (fused small path vs batched kernels)
        assert rel_err(c[c_off[b]:c_off[b + 1]], cs.cpu().numpy()) <= 5e-14, b
        p.destroy()
    bp.destroy()


def test_row_pairs_small_ragged_batch(lc, monkeypatch):
    # the quadrature shape with two rows per lane group (LC_BATCH_ROW_PAIRS=1,
    # used where 2Q splits into whole 16-byte chunks: Q = 16, 32, 48, 64 here,
    # both precisions) against the method oracle and against the one-row
    # shapes (LC_BATCH_ROW_PAIRS=0: another summation order)
    import torch
    banner(f"[gpu] ragged batch of {len(SMALL)}, row pairs")
    funcs = [s[0] for s in SMALL]
    N = [s[1] for s in SMALL]
    M = [s[2] for s in SMALL]
    Q = [s[3] for s in SMALL]
    prec = [s[4] for s in SMALL]
    monkeypatch.setenv("LC_BATCH_ROW_PAIRS", "0")
    bp, arena, c_off = _build(lc, funcs, N, M, Q, prec)
    c1 = bp.execute(arena).cpu().numpy()
    bp.destroy()
    monkeypatch.setenv("LC_BATCH_ROW_PAIRS", "1")
    bp, arena, c_off = _build(lc, funcs, N, M, Q, prec)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c2 = bp.execute(arena, stream=s)   # captured graph
        s.synchronize()
    c2 = c2.cpu().numpy()
    for b, (f, n, m, q, pr) in enumerate(SMALL):
        got = c2[c_off[b]:c_off[b + 1]]
        ref = np.array(oracle.method_coeffs(f, n, expected_grid(m), q), dtype=float)
        if pr == "fp64":
            assert rel_err(got, ref) <= TOL, b
            assert rel_err(got, c1[c_off[b]:c_off[b + 1]]) <= 5e-14, b
        else:
            k = 2 * np.arange(n) + 1
            assert rel_err(got / k, ref / k) <= 1e-7, b
            assert rel_err(got, c1[c_off[b]:c_off[b + 1]]) <= 5e-14, b
    bp.destroy()


def test_graph_replay_and_eager_identical(lc):
    import torch
    banner("[gpu] graph replay / eager / re-capture")
    funcs = [s[0] for s in SMALL]
    N = [s[1] for s in SMALL]
    M = [s[2] for s in SMALL]
    Q = [s[3] for s in SMALL]
    prec = [s[4] for s in SMALL]
    bp, arena, c_off = _build(lc, funcs, N, M, Q, prec)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        outs = []
        for _ in range(3):
            c = torch.full((int(c_off[-1]),), float("nan"), dtype=torch.float64, device="cuda")
            outs.append(bp.execute(arena, c, stream=s))
            s.synchronize()
        bp.set_timing(True)           # eager path (events around the quadrature)
        ce = bp.execute(arena, stream=s)
        s.synchronize()
        ms, cnt = bp.kernel_ms()
        bp.set_timing(False)
        arena2 = arena.clone()        # new pointer: re-capture
        c2 = bp.execute(arena2, stream=s)
        s.synchronize()
    for o in outs[1:] + [ce, c2]:
        assert torch.equal(outs[0], o)
    assert cnt == 1 and ms > 0
    bp.destroy()


def _series_subset_parity(lc, sb, idx, Qfun, resolving):
    import torch
    from workloads.gpu import series_ragged
    B = len(idx)
    N = sb.N[idx]
    M = sb.M[idx]
    Q = np.array([Qfun(int(n)) for n in N], dtype=np.int32)
    coeffs = [sb.coeffs[i] for i in idx]
    bp = lc.plan_batch(N, M, Q, "fp64")
    f_off, x_off, c_off = bp.offsets()
    arena = torch.zeros(int(f_off[-1]) + 256, dtype=torch.uint8, device="cuda")
    series_ragged(coeffs, bp.nodes, x_off, arena, f_off, np.zeros(B, dtype=np.int32))
    c = bp.execute(arena)
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    bp.destroy()
    return N, M, Q, coeffs, c, c_off


def test_uneven_series_resolving_q_exact(lc):
    # random Legendre series of degree N_b - 1 with M_b = 4 N_b >= 2 N_b and
    # Q_b >= N_b / 2: the method is exact, so the batch returns the series'
    # own coefficients
    banner("[gpu] uneven series batch at resolving Q: exact coefficients")
    sb = W.batch_uneven(B=4096)
    rng = np.random.default_rng(33)
    idx = np.sort(rng.choice(4096, 16, replace=False))
    N, M, Q, coeffs, c, c_off = _series_subset_parity(lc, sb, idx, lambda n: n // 2 + 2, True)
    for k in range(len(idx)):
        got = c[c_off[k]:c_off[k + 1]]
        assert rel_err(got, coeffs[k]) <= TOL, (k, int(N[k]))


@pytest.mark.parametrize("prec,pairs", [("fp64", "0"), ("fp64", "1"), ("fp32", None)])
def test_uneven_series_full_batch_stated_q(lc, monkeypatch, prec, pairs):
    # The full 4096-function batch at the stated Q = 48 (under-resolving), in
    # the launch the benchmark times: executed on a side stream, so the
    # captured graph runs (first call captures, the second replays); FP64
    # samples with one row per lane group and with row pairs
    # (LC_BATCH_ROW_PAIRS), FP32 samples with the default (row pairs).
    # Arithmetic parity on 64 seeded members, the longest (N_b = 8191, an FFT
    # of 8192 points in LDS) and the shortest among them, against the method
    # oracle.  Those members are sampled at the oracle's own nodes (rounded
    # to FP64) and the same samples go to both sides, so the comparison is
    # arithmetic only.
    import torch
    from workloads.gpu import series_ragged
    banner(f"[gpu] uneven series batch B=4096, Q=48, {prec}, row pairs {pairs}: 64 members through the captured graph")
    if pairs is None:
        monkeypatch.delenv("LC_BATCH_ROW_PAIRS", raising=False)
    else:
        monkeypatch.setenv("LC_BATCH_ROW_PAIRS", pairs)
    esz, flag = (4, 1) if prec == "fp32" else (8, 0)
    sb = W.batch_uneven(B=4096)
    bp = lc.plan_batch(sb.N, sb.M, sb.Q, prec)
    f_off, x_off, c_off = bp.offsets()
    arena = torch.zeros(int(f_off[-1]) + 256, dtype=torch.uint8, device="cuda")
    series_ragged(sb.coeffs, bp.nodes, x_off, arena, f_off, np.full(4096, flag, dtype=np.int32))
    rng = np.random.default_rng(35)
    pick = set(rng.choice(4096, 62, replace=False).tolist())
    pick |= {int(np.argmax(sb.N)), int(np.argmin(sb.N))}
    pick = np.array(sorted(pick))
    assert pick.size == 64 and max(expected_grid(int(m)) // 4 for m in sb.M[pick]) == 8192
    # oracle nodes of the picked members, sampled by the input generator
    Heff = [expected_grid(int(sb.M[b])) // 2 for b in pick]
    xo = np.zeros(pick.size + 1, dtype=np.int64)
    xo[1:] = np.cumsum([h * 48 for h in Heff])
    xs = torch.empty(int(xo[-1]), dtype=torch.float64, device="cuda")
    for k, b in enumerate(pick):
        X = oracle.abel_node_set(expected_grid(int(sb.M[b])), 48).astype(np.float64).reshape(-1)
        xs[int(xo[k]):int(xo[k + 1])] = torch.from_numpy(X).cuda()
    fo = xo * esz
    tmp = torch.zeros(int(fo[-1]), dtype=torch.uint8, device="cuda")
    series_ragged([sb.coeffs[b] for b in pick], xs, xo, tmp, fo, np.full(pick.size, flag, dtype=np.int32))
    for k, b in enumerate(pick):
        arena[int(f_off[b]):int(f_off[b]) + int(fo[k + 1] - fo[k])] = tmp[int(fo[k]):int(fo[k + 1])]
    # the oracle takes the very samples the kernels read (FP32 ones exactly)
    samples = tmp.view(torch.float32 if prec == "fp32" else torch.float64).cpu().numpy().astype(np.float64)
    del tmp, xs
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c1 = bp.execute(arena, stream=s)
        c2 = torch.full_like(c1, float("nan"))
        bp.execute(arena, c2, stream=s)
        s.synchronize()
    assert torch.equal(c1, c2)
    c = c2.cpu().numpy()
    bp.destroy()
    del arena, c1, c2
    torch.cuda.empty_cache()
    worst = 0.0
    for k, b in enumerate(pick):
        n, Me, H = int(sb.N[b]), expected_grid(int(sb.M[b])), Heff[k]
        sk = samples[int(xo[k]):int(xo[k + 1])].reshape(H, 48)
        ref = np.array(oracle.method_coeffs_from_samples(sk, n, Me, 48), dtype=float)
        got = c[c_off[b]:c_off[b + 1]]
        err = rel_err(got, ref)
        worst = max(worst, err)
        assert err <= TOL, (int(b), n, err)
    banner(f"    64 members (N_b {int(sb.N[pick].min())}..{int(sb.N[pick].max())}): worst rel err {worst:.2e}")


@pytest.mark.parametrize("parts", [1, 2])
def test_short_functions_packed(lc, monkeypatch, parts):
    # many short functions: those of equal FFT length (L <= 256) share
    # workgroups, up to 32 per workgroup; full and partly filled workgroups,
    # every length from 1 to 216 packed, across pipeline parts
    import torch
    monkeypatch.setenv("LC_BATCH_PARTS", str(parts))
    rng = np.random.default_rng(11)
    Ns = [int(n) for n in rng.choice([1, 2, 5, 16, 30, 31, 64, 100, 128, 200], size=150)]
    M = [4 * n for n in Ns]
    fams = [W.GeneratingFunction(0.3), W.Exponential(-1.5), W.Cosine(3.0)]
    funcs = [fams[b % 3] for b in range(len(Ns))]
    prec = ["fp64" if b % 4 else "fp32" for b in range(len(Ns))]
    Q = [24] * len(Ns)
    banner(f"[gpu] {len(Ns)} short functions, {parts} part(s)")
    bp, arena, c_off = _build(lc, funcs, Ns, M, Q, prec)
    c = bp.execute(arena)
    torch.cuda.synchronize()
    c = c.cpu().numpy()
    for b, (f, n, m, pr) in enumerate(zip(funcs, Ns, M, prec)):
        got = c[c_off[b]:c_off[b + 1]]
        ref = np.array(oracle.method_coeffs(f, n, expected_grid(m), 24), dtype=float)
        if pr == "fp64":
            assert rel_err(got, ref) <= TOL, b
        else:
            k = 2 * np.arange(n) + 1
            assert rel_err(got / k, ref / k) <= 1e-7, b
    bp.destroy()


def _four_step_split(L: int) -> tuple[int, int]:
    """The documented four-step split: L1 the largest divisor <= sqrt(L) with
    both factors <= 2048."""
    best, a = 0, 2
    while a * a <= L:
        if L % a == 0 and a <= 2048 and L // a <= 2048:
            best = a
        a += 1
    return best, L // best


def test_long_function_wide_four_step(lc):
    """A function whose FFT has four-step factors above 512 points (M =
    2.2e6: L = 559872 = 729 x 768) beside a short one: the batched four-step
    and the single-function four-step (256-thread blocks at these factors)
    must both give the generating function's t^n."""
    import torch
    from closed_forms import genfn_coeffs
    t = 0.5
    N, M, Q = [2000, 64], [2_200_000, 256], [24, 32]  # Q = 16 leaves the rule's 2e-11 in c_0..c_2
    L1, L2 = _four_step_split(expected_grid(M[0]) // 4)
    assert max(L1, L2) > 512, (L1, L2)
    banner(f"[gpu] batch with a long function: L = {L1} x {L2}")
    funcs = [W.GeneratingFunction(t), W.GeneratingFunction(0.3)]
    bp, arena, c_off = _build(lc, funcs, N, M, Q, ["fp64", "fp64"])
    c = bp.execute(arena).cpu().numpy()
    torch.cuda.synchronize()
    got = c[c_off[0]:c_off[1]]
    exact = np.array(genfn_coeffs(t, N[0]), dtype=float)
    assert float(np.max(np.abs(got - exact))) <= 1e-12
    short = c[c_off[1]:c_off[2]]
    assert float(np.max(np.abs(short - np.array(genfn_coeffs(0.3, N[1]), dtype=float)))) <= 1e-12
    bp.destroy()
    del arena
    p = lc.plan(N[0], M[0], Q[0])
    fx = funcs[0].torch(p.nodes).contiguous()
    cs = p.execute(fx).cpu().numpy()
    torch.cuda.synchronize()
    assert rel_err(got, cs) <= 5e-14
    p.destroy()


def test_fused_small_functions(lc, monkeypatch):
    """The fused one-workgroup path (LC_BATCH_FUSE=1: quadrature rows into
    LDS, then the DST, for functions of at most 2048 rows whose row length
    suits it): FP64 and FP32 samples, Q of 8 to 176 lanes' worth, a Q that
    does not suit it (33, tiled) and a four-step member beside them; equal to
    the method oracle and to the same plan without fusion."""
    import torch
    Ns = [1, 7, 30, 64, 200, 511, 1000, 1024, 300, 5000]
    M = [4, 28, 120, 256, 800, 2044, 4000, 4096, 1200, 40000]
    Q = [2, 16, 48, 48, 24, 176, 48, 64, 33, 48]
    prec = ["fp64", "fp32", "fp64", "fp32", "fp64", "fp64", "fp32", "fp64", "fp64", "fp64"]
    fams = [W.GeneratingFunction(0.4), W.Exponential(1.3), W.Cosine(5.0), W.Rational(3.0)]
    funcs = [fams[b % 4] for b in range(len(Ns))]
    banner(f"[gpu] fused small functions, {len(Ns)} functions")
    out = {}
    for fuse in ("0", "1"):
        monkeypatch.setenv("LC_BATCH_FUSE", fuse)
        monkeypatch.setenv("LC_BATCH_FUSE_HMIN", "2")
        bp, arena, c_off = _build(lc, funcs, Ns, M, Q, prec)
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            c1 = bp.execute(arena, stream=s)
            c2 = torch.full_like(c1, float("nan"))
            bp.execute(arena, c2, stream=s)  # graph replay
            s.synchronize()
        assert torch.equal(c1, c2)
        out[fuse] = c2.cpu().numpy()
        bp.destroy()
    for b, (f, n, m, q, pr) in enumerate(zip(funcs, Ns, M, Q, prec)):
        got, plain = out["1"][c_off[b]:c_off[b + 1]], out["0"][c_off[b]:c_off[b + 1]]
        k = 2 * np.arange(n) + 1
        assert rel_err(got / k, plain / k) <= 1e-13, b
        if n * expected_grid(m) <= 2_000_000:
            ref = np.array(oracle.method_coeffs(f, n, expected_grid(m), q), dtype=float)
            if pr == "fp64":
                assert rel_err(got, ref) <= TOL, b
            else:
                assert rel_err(got / k, ref / k) <= 1e-7, b
