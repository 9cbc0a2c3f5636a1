"""Pins of the oracle's composite Abel rule (breakpoints of f, geometric
grading toward x = 1, per-row node counts for band-limited f) against the
mathematics: the closed-form transforms of P_m (eq. (2.14)), of the
generating function eq. (2.2) and of cos(omega x) (each pinned to mpmath
quadrature of eq. (2.14) here), and the True column of Table 1 for
|x|^{3/2} (the closed form before the table)."""
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
import workloads as W
from closed_forms import abs_pow_coeffs, load_table1, phi_cos, phi_genfn, phi_legendre, phi_quad

LD = np.longdouble
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_closed_forms_vs_mpmath_quadrature():
    mp.mp.dps = 40
    for y in (0.3, 1.9, 3.0):
        t = mp.mpf(0.9)  # the binary value of 0.9, as phi_genfn receives it
        ref = phi_quad(lambda x: 1 / mp.sqrt(1 - 2 * x * t + t * t), y)
        assert abs(phi_genfn(0.9, y) - ref) < mp.mpf(10) ** -20
        ref = phi_quad(lambda x: mp.cos(37 * x), y)
        assert abs(phi_cos(37, y) - ref) < mp.mpf(10) ** -20


def test_ladder():
    # multiples of 8 up to 128, then 16 steps per octave (at most 6.25% over)
    assert [oracle.abel_rule_ladder(n) for n in (1, 8, 9, 128, 129, 136, 137, 255, 256, 257, 8193)] == \
        [8, 8, 16, 128, 136, 136, 144, 256, 256, 272, 8704]
    for n in range(1, 20000, 7):
        v = oracle.abel_rule_ladder(n)
        assert n <= v <= max(n + 7, int(n * 1.0625) + 1)


def test_cuts_map_breakpoints_and_grading():
    rule = {"q": 8, "breaks": [-0.25, 0.0, 0.6], "grade_ratio": 0.2, "grade_levels": 3}
    for y in (0.7, 1.9, 3.1):
        s = np.sin(LD(y) / 2)
        c = np.cos(LD(y))
        es = oracle.abel_rule_cuts(s, rule)
        # every breakpoint inside (cos y, 1) gives a cut with x(t) = b
        inside = [b for b in rule["breaks"] if c < b < 1]
        xs = [1 - 2 * s * s * e * (2 - e) for e in es]
        for b in inside:
            assert min(abs(x - LD(b)) for x in xs) < 1e-17
        # the grading cuts 1 - t = sigma^k
        for k in (1, 2, 3):
            assert min(abs(e - LD(0.2) ** k) for e in es) < 1e-18
        assert len(es) == len(inside) + 3
        assert all(es[i] > es[i + 1] for i in range(len(es) - 1))


@pytest.mark.parametrize("m", [0, 7, 20])
def test_composite_rule_exact_for_legendre(m):
    # each panel's rule is exact for f of degree m when q >= m + 1 (full
    # q-point panels integrate degree 2m in t; the half rule degree 4q - 1)
    rule = {"q": m + 1 + (m + 1) % 2, "breaks": [0.0, -0.5], "grade_ratio": 0.15, "grade_levels": 4}
    cm = np.zeros(m + 1)
    cm[m] = 1.0
    f = lambda x: npleg.legval(np.asarray(x, dtype=np.float64), cm)
    y = np.linspace(0.05, np.pi, 17, dtype=LD)
    got = np.array(oracle.abel_phi_rule(f, y, rule), dtype=float)
    ref = np.array([float(phi_legendre(m, float(v))) for v in y])
    assert np.max(np.abs(got - ref)) < 5e-15


def test_grading_resolves_near_singular_generating_function():
    # t = 0.999: singular at x = (1 + t^2)/(2t) = 1 + 5e-7.  Geometric panels
    # toward x = 1 reach ~1e-9 with ~170 nodes per row where the uniform
    # rule with 512 nodes is off by ~1e-4
    t = 0.999
    f = W.GeneratingFunction(t)
    graded = {"q": 24, "grade_ratio": 0.15, "grade_levels": 6}
    ys = np.array([0.5, 1.3, 2.2, 3.0, np.pi], dtype=LD)
    g = np.array(oracle.abel_phi_rule(f, ys, graded), dtype=float)
    u = np.array(oracle.abel_phi(f, ys, 512), dtype=float)
    ref = np.array([float(phi_genfn(t, float(v))) for v in ys])
    err_g = np.max(np.abs(g - ref) / np.abs(ref))
    err_u = np.max(np.abs(u - ref) / np.abs(ref))
    assert err_g < 1e-8, err_g
    assert err_u > 100 * err_g


def test_band_rule_resolves_cosine_with_fewer_nodes():
    # cos(D x) needs about D s^2 / 2 nodes in the row with s = sin(y/2)
    D = 1024
    rule = {"q": 8, "band": D, "q_max": 4096}
    f = W.Cosine(D)
    ys = np.array([0.02, 0.1, 0.4, 1.0, 2.0, 2.8, np.pi], dtype=LD)
    got = np.array(oracle.abel_phi_rule(f, ys, rule), dtype=float)
    ref = np.array([float(phi_cos(D, float(v))) for v in ys])
    assert np.max(np.abs(got - ref)) < 1e-13
    # the row counts follow D s^2 / 2 (plus the stated pad), half the
    # uniform D / 2 + pad on average over the grid
    M = 2048
    n_rule = oracle.abel_rule_node_count(M, rule)
    q_uniform = oracle.abel_rule_row_q(LD(1), rule)          # the count at y = pi
    assert n_rule < 0.6 * (M // 2) * q_uniform


def test_breakpoint_reaches_table1_error_level():
    # |x|^{3/2} (Table 1): a breakpoint at x = 0 brings the method to the
    # paper's error level (its Error column is 2.7e-12 .. 1.6e-9); one global
    # Gauss rule is stuck near 1e-7 by the kink inside [cos y, 1]
    ns, vals = load_table1(os.path.join(GOLDEN, "table1_abs_x_3_2.txt"))
    N = max(ns) + 2
    true = abs_pow_coeffs(N, Fraction(3, 2))
    f = W.AbsPower(1.5)
    M = 4096
    c_bp = oracle.method_coeffs_rule(f, N, M, {"q": 64, "breaks": [0.0]})
    c_gl = oracle.method_coeffs(f, N, 1024, 256)
    err_bp = max(abs(float(c_bp[n]) - float(true[n])) for n in ns)
    err_gl = max(abs(float(c_gl[n]) - float(true[n])) for n in ns)
    assert err_bp < 2e-9, err_bp
    assert err_gl > 30 * err_bp
    # and the printed True values themselves (20 digits, truncated) agree
    # with the closed form
    for n, v in zip(ns, vals):
        assert abs(Fraction(v) - true[n]) < Fraction(1, 10 ** 19)
