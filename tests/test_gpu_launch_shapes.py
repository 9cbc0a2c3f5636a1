"""GPU checks of every launch shape of the uniform Abel reductions.

The autotuner times all supported shapes of the single and batched
quadrature reductions but only the chosen one reaches a caller.  Here each
shape is forced through the autotuner's cache file (its last entry for a
plan wins) and executed: exact-fit variants (weights in registers, rows
unrolled), also over row pairs (two rows per lane group),
one-chunk-per-lane variants (rows shorter than a lane group, the spare lanes
idle) and generic variants (any Q), each with a one-block grid (one
block strides over every row), a few blocks and more blocks than rows.
Every result must equal the default shape's up to summation order, and the
single FP64 plan also matches the method oracle.  The DST workgroup sizes of
single plans are forced the same way over power-of-two FFT lengths.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from helpers import banner, expected_grid, rel_err

pytestmark = pytest.mark.gpu
QS = (48, 20)  # 20: rows of 5 (FP32) or 10 (FP64) 16-byte chunks
GRIDS = (1, 5, 1 << 20)
FIT_KEYS = {17, 18, 20, 33, 34, 36, 49, 50, 65, 66, 97, 129}  # 16 cpl + unroll of the built variants


@pytest.fixture(scope="module")
def lc():
    import torch
    import paper_1106_0463_amd as lc
    torch.cuda.set_device(0)
    return lc


def shapes(prec: str, q: int):
    """(vec, G, cpl, unroll, rows per lane group) of every reduction the
    library accepts for q."""
    out = []
    vfit = 2 if prec == "fp64" else 4
    for rpg in (1, 2):
        for G in (4, 8, 16):
            for cpl in (1, 2, 3, 4, 6, 8):
                for u in (1, 2, 4):
                    if G * cpl * vfit == rpg * q and cpl * 16 + u in FIT_KEYS:
                        out.append((vfit, G, cpl, u, rpg))
    nch = q // vfit  # one 16-byte chunk per lane, lanes past nch idle
    for G in (8, 16, 32, 64):
        if q % vfit == 0 and G < 2 * nch <= 2 * G:
            out.extend((vfit, G, -1, u, 1) for u in (1, 2, 4, 8))
    for vec in (1, 2):
        for G in (4, 8, 16, 32, 64):
            if q % vec == 0 and (vec == 1 or G >= 16):
                out.append((vec, G, 0, 1, 1))
    return out


def _last_entry(path, kind):
    lines = [ln.rstrip("\n") for ln in open(path) if f"|{kind}|" in ln]
    assert lines, f"no {kind} entry in the cache"
    key, val = lines[-1].split("\t")
    return key, val.split()


def _force(path, key, tokens):
    with open(path, "a") as fh:
        fh.write(key + "\t" + " ".join(str(t) for t in tokens) + "\n")


def _assert_taken(path, kind, tokens):
    """A cache entry the library rejects is tuned again and a new entry
    appended: the forced one must still be the last."""
    _, last = _last_entry(path, kind)
    assert last == [str(t) for t in tokens], ("forced shape not taken", tokens, last)


@pytest.mark.parametrize("Q", QS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_single_shapes(lc, tmp_path, monkeypatch, prec, Q):
    import torch
    cache = str(tmp_path / "tune.txt")
    monkeypatch.setenv("LC_AUTOTUNE_CACHE", cache)
    N, M = 300, 2400  # 460 KB of FP64 samples: past the fused single-workgroup path
    f = W.Exponential(-2.5)
    p = lc.plan(N, M, Q, precision=prec)
    fx = f.torch(p.nodes).contiguous()
    if prec == "fp32":
        fx = fx.float().contiguous()
    ref = p.execute(fx).cpu().numpy()
    p.autotune()
    key, tok = _last_entry(cache, "single")
    assert tok[0] == "quad" and tok[8] == "dst" and tok[-2] == "fused"
    tok[-1] = "0"  # the reduction kernel, not the fused small path
    if prec == "fp64":
        Me = expected_grid(M)
        want = np.array(oracle.method_coeffs(f, N, Me, Q), dtype=float)
        assert rel_err(ref, want) <= 1e-12
    worst = 0.0
    cases = [(s, g) for s in shapes(prec, Q) for g in GRIDS]
    banner(f"[gpu] single {prec} Q={Q}: {len(cases)} reduction shapes x grids")
    for (vec, G, cpl, u, rpg), grid in cases:
        forced = ["quad", vec, G, cpl, u, 256, grid, rpg] + tok[8:]
        _force(cache, key, forced)
        p.autotune()
        _assert_taken(cache, "single", forced)
        got = p.execute(fx).cpu().numpy()
        torch.cuda.synchronize()
        e = rel_err(got, ref)
        worst = max(worst, e)
        assert e <= 1e-13, (vec, G, cpl, u, grid, e)
    banner(f"    worst difference to the default shape {worst:.2e}")
    p.destroy()


@pytest.mark.parametrize("Q", QS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_shapes(lc, tmp_path, monkeypatch, prec, Q):
    import torch
    from workloads.gpu import fill_closed_form_arena
    cache = str(tmp_path / "tune.txt")
    monkeypatch.setenv("LC_AUTOTUNE_CACHE", cache)
    Ns = [40, 300, 77, 1000, 5]
    Ms = [96, 1200, 200, 2400, 10]
    funcs = [W.Exponential(a) for a in (-1.0, 2.0, -3.5, 0.5, 1.5)]
    bp = lc.plan_batch(Ns, Ms, [Q] * len(Ns), prec)
    f_off, x_off, c_off = bp.offsets()
    H = [expected_grid(m) // 2 for m in Ms]
    arena = torch.zeros(int(f_off[-1]) + 256, dtype=torch.uint8, device="cuda")
    fill_closed_form_arena(bp.nodes, arena, x_off, f_off, H, [Q] * len(Ns), funcs, [prec == "fp32"] * len(Ns))
    ref = bp.execute(arena).cpu().numpy()
    bp.autotune()
    key, tok = _last_entry(cache, "batch2")
    assert tok[0] == "1"  # one (Q, precision) class: its seven shape numbers follow
    worst = 0.0
    cases = [(s, g) for s in shapes(prec, Q) for g in GRIDS]
    banner(f"[gpu] batch {prec} Q={Q}: {len(cases)} reduction shapes x grids")
    for (vec, G, cpl, u, rpg), grid in cases:
        forced = ["1", vec, G, cpl, u, 256, grid, rpg] + tok[8:]
        _force(cache, key, forced)
        bp.autotune()
        _assert_taken(cache, "batch2", forced)
        got = bp.execute(arena).cpu().numpy()
        torch.cuda.synchronize()
        e = rel_err(got, ref)
        worst = max(worst, e)
        assert e <= 1e-13, (vec, G, cpl, u, rpg, grid, e)
    banner(f"    worst difference to the default shape {worst:.2e}")
    bp.destroy()


@pytest.mark.parametrize("L", [64, 128, 256, 512, 1024, 2048, 4096, 8192, 80, 240, 640, 1920, 5120, 7680])
def test_single_dst_threads(lc, tmp_path, monkeypatch, L):
    """Every DST workgroup size T with L <= 8 T, forced through the cache, on
    an FFT of length L = H/2: power-of-two lengths 2T, 4T and 8T take the
    compile-time Stockham passes, the others (and the lengths 5 2^a and
    15 2^a, with their radix-5 pass) the run-time schedule.  All must give
    the default shape's coefficients up to rounding order, and the method
    oracle's."""
    import torch
    cache = str(tmp_path / "tune.txt")
    monkeypatch.setenv("LC_AUTOTUNE_CACHE", cache)
    M, N, q = 4 * L, min(200, L), 16
    f = W.Exponential(-2.5)
    p = lc.plan(N, M, q)
    assert p.info["M_eff"] == M and p.info["H"] == 2 * L
    fx = f.torch(p.nodes).contiguous()
    ref = p.execute(fx).cpu().numpy()
    want = np.array(oracle.method_coeffs(f, N, M, q), dtype=float)
    assert rel_err(ref, want) <= 1e-12
    p.autotune()
    key, tok = _last_entry(cache, "single")
    assert tok[8] == "dst" and tok[-2] == "fused"
    tok[-1] = "0"  # the DST kernel, not the fused small path
    sizes = [T for T in (64, 128, 256, 512, 1024) if L <= 8 * T]
    banner(f"[gpu] single DST L={L}: workgroup sizes {sizes}")
    for T in sizes:
        forced = tok[:9] + [str(T)] + tok[10:]
        _force(cache, key, forced)
        p.autotune()
        _assert_taken(cache, "single", forced)
        got = p.execute(fx).cpu().numpy()
        torch.cuda.synchronize()
        e = rel_err(got, ref)
        assert e <= 1e-13, (T, e)
        assert rel_err(got, want) <= 1e-12, T
    p.destroy()
