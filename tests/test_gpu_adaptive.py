"""GPU checks of adaptive plans (composite Abel rule: breakpoints of f,
geometric grading toward x = 1, per-row node counts), against the oracle's
independent implementation of the same rule (arithmetic parity: both sides
sample f at their own correctly rounded FP64 nodes) and against the truth:

* |x|^{3/2} with a breakpoint at x = 0: Table 1's True column at the
  paper's error level (its Error column: 2.7e-12 .. 1.6e-9);
* the generating function eq. (2.2) at t = 0.999 with grading: c_n = t^n;
* cos(omega x) with the band rule: the closed form of its coefficients;
* a rule without cuts or band equals the uniform plan (same Gauss rule);
* rows of exactly 16 panels, and plans that mix rows of at most 16 panels
  (one run of chunks per row) with rows of more (panel by panel).
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads as W
from closed_forms import abs_pow_coeffs, cos_coeff, load_table1
from helpers import banner, rel_err

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lc():
    import torch
    import paper_1106_0463_amd as lc
    torch.cuda.set_device(0)
    return lc


def _run(lc, f, N, M, rule, precision="fp64"):
    import torch
    p = lc.plan_adaptive(N, M, precision=precision, **rule)
    x = p.nodes
    fx = f.torch(x).contiguous()
    if precision == "fp32":
        fx = fx.float().contiguous()
    c = p.execute(fx)
    torch.cuda.synchronize()
    out = c.cpu().numpy()
    info = p.info
    p.destroy()
    return out, info


def _orule(rule):
    return {k: v for k, v in rule.items()}


def test_nodes_match_oracle_rule(lc):
    # the nodes of every row, in the documented layout, against the oracle's
    # own construction (long double, rounded to FP64)
    import torch
    banner("[gpu] adaptive nodes vs oracle rule")
    rule = dict(q=8, breaks=(0.0, -0.6), grade_ratio=0.2, grade_levels=3)
    M = 64
    p = lc.plan_adaptive(16, M, **rule)
    x = p.nodes.cpu().numpy()
    p.destroy()
    H = M // 2
    LD = np.longdouble
    pos = same = total = 0
    for j in range(1, H + 1):
        s = np.sin(oracle.method.PI * j / (2 * H))
        q = oracle.abel_rule_row_q(s, rule)
        cuts = oracle.abel_rule_cuts(s, rule)
        T, _ = oracle.gauss_legendre(2 * q)
        tau, _ = oracle.gauss_legendre(q)
        bounds = [LD(1)] + cuts + [LD(0)]
        panels = [bounds[1] + (1 - bounds[1]) * (1 - T[:q])]
        for k in range(1, len(bounds) - 1):
            h = (bounds[k] - bounds[k + 1]) / 2
            panels.append(bounds[k + 1] + h * (1 - tau[::-1]))
        for e in panels:
            ref_ld = 1 - 2 * s * s * e * (2 - e)
            ref = ref_ld.astype(np.float64)
            qp = (len(e) + 3) // 4 * 4
            got = x[pos:pos + qp]
            # correctly rounded on both sides: equal but for rare near-ties,
            # where the oracle's long-double rounding may land one ulp away,
            # and near x = 0, where its long-double evaluation of
            # 1 - 2 s^2 (1 - t^2) carries ~1e-19 of cancellation error
            assert np.all(np.abs(got[:len(e)] - ref) <= np.spacing(np.abs(ref)) + 4e-19), j
            same += int(np.sum(got[:len(e)] == ref))
            total += len(e)
            assert np.all(got[len(e):] == got[len(e) - 1])
            pos += qp
    assert pos == x.size
    assert same >= 0.99 * total


@pytest.mark.parametrize("N,M,q", [(1, 8, 1), (33, 200, 7), (500, 2000, 24), (3000, 70000, 16)])
def test_rule_without_cuts_equals_uniform_plan(lc, N, M, q):
    import torch
    banner(f"[gpu] adaptive (no cuts) vs uniform plan N={N} M={M} q={q}")
    f = W.Exponential(1.7)
    ca, info = _run(lc, f, N, M, dict(q=q))
    p = lc.plan(N, M, q)
    cu = p.execute(f.torch(p.nodes).contiguous())
    torch.cuda.synchronize()
    cu = cu.cpu().numpy()
    p.destroy()
    assert info["samples"] == info["H"] * ((q + 3) // 4 * 4)
    # same nodes (up to near-ties) and weights; only the summation order
    # differs, which moves the rounding noise of the tail (~1e-14 max|c|)
    assert rel_err(ca, cu) <= 5e-14


def test_breakpoint_table1(lc):
    banner("[gpu] adaptive |x|^{3/2}, breakpoint at 0 (Table 1)")
    ns, _ = load_table1(os.path.join(GOLDEN, "table1_abs_x_3_2.txt"))
    N, M = 32, 4096
    rule = dict(q=64, breaks=(0.0,))
    got, _ = _run(lc, W.AbsPower(1.5), N, M, rule)
    ref = np.array(oracle.method_coeffs_rule(W.AbsPower(1.5), N, M, _orule(rule), fp64_nodes=True), dtype=float)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    true = np.array([float(v) for v in abs_pow_coeffs(N, Fraction(3, 2))])
    err_true = max(abs(got[n] - true[n]) for n in ns)
    banner(f"    vs oracle {err:.2e}; max |c - true| over Table 1's n: {err_true:.2e}")
    assert err <= 1e-13
    assert err_true <= 2e-9


def test_grading_generating_function(lc):
    banner("[gpu] adaptive generating function t=0.999, graded")
    t, N, M = 0.999, 256, 32768
    rule = dict(q=16, grade_ratio=0.15, grade_levels=8)
    f = W.GeneratingFunction(t)
    got, info = _run(lc, f, N, M, rule)
    ref = np.array(oracle.method_coeffs_rule(f, N, M, _orule(rule), fp64_nodes=True), dtype=float)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    err_true = np.max(np.abs(got - t ** np.arange(N)))
    banner(f"    vs oracle {err:.2e}; vs t^n {err_true:.2e}; {info['samples'] / info['H']:.0f} nodes/row")
    assert err <= 1e-12
    assert err_true <= 1e-9


def test_band_rule_cosine(lc):
    banner("[gpu] adaptive cos(2048 x), band rule")
    om, N, M = 2048, 2048, 8192
    rule = dict(q=8, band=om, q_max=4096)
    f = W.Cosine(om)
    got, info = _run(lc, f, N, M, rule)
    ref = np.array(oracle.method_coeffs_rule(f, N, M, _orule(rule), fp64_nodes=True), dtype=float)
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref)) / scale
    idx = np.arange(0, N, 97)
    true = np.array([float(cos_coeff(om, int(n))) for n in idx])
    err_true = np.max(np.abs(got[idx] - true)) / scale
    uniform = (M // 2) * oracle.abel_rule_row_q(np.longdouble(1), rule)
    banner(f"    vs oracle {err:.2e}; vs closed form {err_true:.2e}; samples {info['samples']} "
           f"({info['samples'] / uniform:.2f} of the uniform rule)")
    assert err <= 1e-12
    assert err_true <= 1e-12
    assert info["samples"] < 0.6 * uniform


def test_fp32_samples(lc):
    banner("[gpu] adaptive FP32 samples vs FP64")
    N, M = 512, 4096
    rule = dict(q=32, breaks=(0.0, 0.5), grade_ratio=0.3, grade_levels=2)
    f = W.AbsPower(1.5)
    c64, _ = _run(lc, f, N, M, rule)
    c32, info = _run(lc, f, N, M, rule, precision="fp32")
    n = np.arange(N)
    E_a = np.max(np.abs((c32 - c64) / (2 * n + 1))) / np.max(np.abs(c64 / (2 * n + 1)))
    banner(f"    E_a(fp32 vs fp64) {E_a:.2e}")
    assert E_a <= 1e-7


def _panel_counts(M, rule):
    H = M // 2
    return [1 + len(oracle.abel_rule_cuts(np.sin(oracle.method.PI * j / (2 * H)), rule)) for j in range(1, H + 1)]


@pytest.mark.parametrize("rule,mixed", [
    (dict(q=8, grade_ratio=0.5, grade_levels=15), False),
    (dict(q=8, breaks=(0.0, 0.3, -0.5, 0.7, 0.9), grade_ratio=0.5, grade_levels=12), True),
])
def test_many_panels(lc, rule, mixed):
    N, M = 200, 1024
    counts = _panel_counts(M, rule)
    banner(f"[gpu] adaptive {min(counts)}..{max(counts)} panels per row, |x|^(3/2)")
    if mixed:
        assert min(counts) <= 16 < max(counts)
    else:
        assert min(counts) == max(counts) == 16
    f = W.AbsPower(1.5)
    got, info = _run(lc, f, N, M, rule)
    ref = np.array(oracle.method_coeffs_rule(f, N, M, _orule(rule), fp64_nodes=True), dtype=float)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    banner(f"    vs oracle {err:.2e}")
    assert err <= 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("gmax", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("gmul", [0, 1])
def test_launch_shapes(lc, monkeypatch, gmax, gmul, prec):
    # every lane count of the reductions, with one row per lane group and
    # with a grid stride (a group then walks several rows and reuses its
    # panel-table slot), on rows of mixed lengths (about 200 to 1000 samples:
    # each cap up to 64 lanes is used) and 13 to 18 panels (both the flattened
    # and the panel-by-panel reduction)
    monkeypatch.setenv("LC_AQUAD_GMAX", str(gmax))
    monkeypatch.setenv("LC_AQUAD_GMUL", str(gmul))
    banner(f"[gpu] adaptive {prec} launch shape: lane cap {4 << gmax}, "
           f"grid {'one row per group' if gmul == 0 else 'stride'}")
    N, M = 300, 2048
    rule = dict(q=8, band=1024.0, q_max=1024, breaks=(0.0, 0.3, -0.5, 0.7, 0.9), grade_ratio=0.5, grade_levels=12)
    f = W.AbsPower(1.5)
    got, info = _run(lc, f, N, M, rule, precision=prec)
    ref = np.array(oracle.method_coeffs_rule(f, N, M, _orule(rule), fp64_nodes=True), dtype=float)
    if prec == "fp64":
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= 1e-13
    else:  # FP32 samples: the mixed class, in a_n = c_n / (2n + 1)
        k = 2 * np.arange(N) + 1
        err = np.max(np.abs(got / k - ref / k)) / np.max(np.abs(ref / k))
        assert err <= 1e-7
    banner(f"    vs oracle {err:.2e}")
