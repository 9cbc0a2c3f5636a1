"""Pins of the definition oracle (eq. (2.3) by brute-force quadrature)
against values fixed by the paper and by the mathematics, independently of
the oracle's own code."""
import os
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
import workloads as W
from closed_forms import (abs_pow_coeffs, coeff_quad, cos_coeffs, exp_coeffs,
                          genfn_coeffs, load_table1)

LD = np.longdouble
HERE = os.path.dirname(os.path.abspath(__file__))


def _f(v):
    return np.array([float(t) for t in v])


# ---------------------------------------------------------------- GL rule --

def test_gauss_legendre_textbook_5pt():
    # classical closed form of the 5-point rule
    x, w = oracle.gauss_legendre(5)
    r = np.sqrt(10.0 / 7.0)
    xs = sorted([0.0, np.sqrt(5 - 2 * r) / 3, -np.sqrt(5 - 2 * r) / 3,
                 np.sqrt(5 + 2 * r) / 3, -np.sqrt(5 + 2 * r) / 3], reverse=True)
    ws = {0.0: 128 / 225}
    wi = (322 + 13 * np.sqrt(70)) / 900
    wo = (322 - 13 * np.sqrt(70)) / 900
    assert np.allclose(np.array(x, dtype=float), xs, atol=1e-15, rtol=0)
    assert np.allclose(np.array(w, dtype=float), [wo, wi, ws[0.0], wi, wo],
                       atol=1e-15, rtol=0)


@pytest.mark.parametrize("K", [1, 2, 7, 20, 64])
def test_gauss_legendre_monomial_exactness(K):
    # sum w x^m = integral_{-1}^1 x^m dx for m <= 2K-1, exactly in rationals
    x, w = oracle.gauss_legendre(K)
    for m in range(2 * K):
        exact = 0.0 if m % 2 else 2.0 / (m + 1)
        got = float(np.sum(w * x ** m))
        assert abs(got - exact) < 5e-17 * K, (K, m, got, exact)
    # for m = 2K the error is the textbook remainder
    #   integral - rule = 2^{2K+1} (K!)^4 / ((2K+1) ((2K)!)^2)
    if K <= 20:
        from math import factorial
        got = np.sum(w * x ** (2 * K))
        rem = Fraction(2 ** (2 * K + 1) * factorial(K) ** 4,
                       (2 * K + 1) * factorial(2 * K) ** 2)
        diff = LD(2) / LD(2 * K + 1) - got
        assert abs(float(diff) / float(rem) - 1.0) < 1e-6


def test_gauss_legendre_large_matches_mpmath_nodes():
    # spot-check nodes of a large rule against mpmath root finding
    K = 1000
    x, w = oracle.gauss_legendre(K)
    mp.mp.dps = 40
    for k in (0, 1, 250, 499):
        # distance to the true zero = one Newton step computed in mpmath
        num, den = LD(x[k]).as_integer_ratio()
        xk = mp.mpf(num) / den
        pk = mp.legendre(K, xk)
        dpk = K * (xk * pk - mp.legendre(K - 1, xk)) / (xk * xk - 1)
        assert abs(pk / dpk) < 1e-18, (k, pk / dpk)
        # weight 2 / ((1 - x^2) P_K'(x)^2) at the true zero (Newton-refined
        # in mpmath); the long-double recurrence leaves ~1e-15 relative at
        # the outermost nodes
        r = xk
        for _ in range(2):
            pr = mp.legendre(K, r)
            r = r - pr / (K * (r * pr - mp.legendre(K - 1, r)) / (r * r - 1))
        pr = mp.legendre(K, r)
        dpr = K * (r * pr - mp.legendre(K - 1, r)) / (r * r - 1)
        wref = 2 / ((1 - r * r) * dpr * dpr)
        assert abs(float(w[k]) / float(wref) - 1.0) < 1e-14, k
    assert abs(float(np.sum(w)) - 2.0) < 1e-16


def test_gauss_legendre_converges_for_every_size():
    # odd and even K, small to large: a valid rule (nodes strictly inside
    # (-1, 1), decreasing, symmetric; weights positive, summing to 2)
    for K in list(range(1, 160)) + [957, 1001, 4097, 20000]:
        x, w = oracle.gauss_legendre(K)
        assert np.all(np.diff(x) < 0) and x[0] < 1 and x[-1] > -1
        assert np.all(w > 0) and abs(float(np.sum(w)) - 2.0) < 1e-15
        assert np.all(x + x[::-1] == 0)


# --------------------------------------------------------- fixed cases ----

@pytest.mark.parametrize("m", [0, 1, 5, 40, 63])
def test_legendre_polynomial_gives_delta(m):
    # f = P_m (evaluated with numpy's float64 legval) => c_n = delta_{nm}
    cm = np.zeros(m + 1)
    cm[m] = 1.0
    f = lambda x: npleg.legval(np.asarray(x, dtype=np.float64), cm)
    c = oracle.legendre_coeffs(f, 80, 80)
    e = np.zeros(80)
    e[m] = 1.0
    assert np.max(np.abs(np.array(c, dtype=float) - e)) < 5e-15


@pytest.mark.parametrize("t", [0.1, 0.5, 0.9])
def test_generating_function_gives_powers(t):
    # eq. (2.2): c_n = t^n
    N = 96
    K = 512 if t < 0.9 else 1024
    c = oracle.legendre_coeffs(W.GeneratingFunction(t), N, K)
    ref = np.array([float(v) for v in genfn_coeffs(t, N)])
    # long-double rounding of the sum, amplified by (n + 1/2)
    assert np.max(np.abs(np.array(c, dtype=float) - ref)) < 5e-16


@pytest.mark.parametrize("a", [1.0, -7.5, 20.0, 0.0])
def test_exponential_gives_spherical_bessel(a):
    N = 64
    c = oracle.legendre_coeffs(W.Exponential(a), N, 128)
    ref = _f(exp_coeffs(a, N))
    scale = max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(np.array(c, dtype=float) - ref)) < 2e-16 * scale * 8


def test_cosine_gives_spherical_bessel():
    N, omega = 200, 64.0
    c = oracle.legendre_coeffs(W.Cosine(omega), N, 400)
    ref = _f(cos_coeffs(omega, N))
    assert np.max(np.abs(np.array(c, dtype=float) - ref)) < 1e-15


def test_abs_pow_closed_form_matches_table1_true_column():
    # the closed form reproduces every printed digit (the table truncates)
    ns, vals = load_table1(os.path.join(HERE, "golden", "table1_abs_x_3_2.txt"))
    cf = abs_pow_coeffs(31)
    for n, v in zip(ns, vals):
        printed = Fraction(v)
        assert abs(cf[n] - printed) < Fraction(1, 10 ** 20), (n, v)


def test_oracle_abs_pow_matches_table1_true_column():
    # |x|^{3/2} with a breakpoint at its kink; Table 1 True column
    ns, vals = load_table1(os.path.join(HERE, "golden", "table1_abs_x_3_2.txt"))
    c = oracle.legendre_coeffs_piecewise(W.AbsPower(1.5), 32, 3000, [0.0])
    for n, v in zip(ns, vals):
        assert abs(float(c[n] - LD(v))) < 2e-16, (n, float(c[n]), v)
    for n in range(1, 32, 2):
        assert abs(float(c[n])) < 1e-17


def test_reconstruction_of_polynomial():
    # eq. (2.1): sum c_n P_n reproduces f for a polynomial of degree 12
    coef = np.random.default_rng(11).standard_normal(13)
    f = lambda x: npleg.legval(np.asarray(x, dtype=np.float64), coef)
    c = oracle.legendre_coeffs(f, 13, 16)
    xs = np.linspace(-1, 1, 41)
    rec = np.array(oracle.legendre_eval(c, xs), dtype=float)
    assert np.max(np.abs(rec - f(xs))) < 1e-14
    assert np.max(np.abs(np.array(c, dtype=float) - coef)) < 1e-14


def test_brute_force_mpmath_rational():
    # f = (1+x)/(gamma^2+x^2), gamma = 0.5: mpmath adaptive quadrature
    gamma = 0.5
    f = W.Rational(gamma)
    c = oracle.legendre_coeffs(f, 11, 256)
    mp.mp.dps = 30
    fm = lambda x: (1 + x) / (mp.mpf(gamma) ** 2 + x * x)
    for n in range(11):
        ref = coeff_quad(fm, n)
        assert abs(float(c[n]) - float(ref)) < 1e-15 * max(1.0, abs(float(ref)))


def test_planted_mistakes_are_caught():
    # A dropped (n + 1/2) factor or a sign slip in the recurrence would move
    # these values by O(1); assert the closed forms are far from such variants.
    c = np.array(oracle.legendre_coeffs(W.GeneratingFunction(0.5), 8, 64), dtype=float)
    ref = 0.5 ** np.arange(8)
    assert np.max(np.abs(c - ref)) < 1e-16
    assert np.max(np.abs(c / (np.arange(8) + 0.5) - ref)) > 0.1


@pytest.mark.parametrize("a", [-20.0, -3.5, 0.7, 13.0, 20.0])
def test_exp_closed_form_fast_matches_mpmath(a):
    # the float64 backward-recurrence closed form of e^{ax} used for long
    # coefficient vectors, against mpmath's Bessel function I_{n+1/2}
    from closed_forms import exp_coeffs, exp_coeffs_fast
    N = 90
    ref = np.array([float(v) for v in exp_coeffs(a, N)])
    got = exp_coeffs_fast(a, N)
    assert np.max(np.abs(got - ref)) <= 2e-16 * np.max(np.abs(ref))
    nz = np.abs(ref) > 1e-280
    assert np.max(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])) <= 1e-14
    long = exp_coeffs_fast(a, 70000)
    assert np.array_equal(long[:N], got) and np.all(long[700:] == 0.0)


def test_exp_closed_form_many_matches_single():
    from closed_forms import exp_coeffs_fast, exp_coeffs_many
    a = np.array([-20.0, -7.25, -0.3, 0.0, 1.0, 19.99])
    many = exp_coeffs_many(a, top=200)
    for k, ak in enumerate(a):
        one = exp_coeffs_fast(ak, 201)
        assert np.max(np.abs(many[k] - one)) <= 4e-16 * np.max(np.abs(one)), ak
