"""Pins of the method oracle (the paper's discretized steps) against the
mathematics: mpmath quadrature of the Abel-type integral eq. (2.14), the
closed-form transform of P_m, exactness of the trapezoid rule for
trigonometric polynomials, polynomial exactness end to end and the exact
aliasing law of the M-point grid."""
import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
import workloads as W
from closed_forms import phi_legendre, phi_quad

LD = np.longdouble


@pytest.mark.parametrize("m", [0, 1, 4, 17])
def test_phi_of_legendre_closed_form_vs_mpmath(m):
    # the closed form phi_{P_m}(y) = 2 sin((m+1/2) y)/(2m+1) against direct
    # tanh-sinh quadrature of eq. (2.14)
    mp.mp.dps = 50
    for y in (0.3, 1.7, 3.0):
        ref = phi_quad(lambda x: mp.legendre(m, x), y)
        assert abs(ref - phi_legendre(m, y)) < mp.mpf(10) ** -25


@pytest.mark.parametrize("m", [0, 3, 30])
def test_abel_phi_of_legendre(m):
    # eq. (2.14) by the oracle's Abel rule with 2Q-1 >= m is exact
    cm = np.zeros(m + 1)
    cm[m] = 1.0
    f = lambda x: npleg.legval(np.asarray(x, dtype=np.float64), cm)
    y = np.linspace(0.0, np.pi, 33, dtype=LD)
    got = np.array(oracle.abel_phi(f, y, Q=(m + 2) // 2 + 1), dtype=float)
    ref = np.array([float(phi_legendre(m, float(v))) for v in y])
    assert np.max(np.abs(got - ref)) < 5e-15


@pytest.mark.parametrize("fam", ["genfn", "exp", "rational"])
def test_abel_phi_vs_mpmath_quadrature(fam):
    mp.mp.dps = 30
    if fam == "genfn":
        f, fm, Q = W.GeneratingFunction(0.6), (lambda x: 1 / mp.sqrt(1 - 2 * x * mp.mpf(0.6) + mp.mpf(0.36))), 48
    elif fam == "exp":
        f, fm, Q = W.Exponential(-3.0), (lambda x: mp.exp(-3 * x)), 24
    else:
        f, fm, Q = W.Rational(2.0), (lambda x: (1 + x) / (4 + x * x)), 24
    ys = [0.05, 0.9, 2.2, np.pi]
    got = np.array(oracle.abel_phi(f, np.array(ys, dtype=LD), Q), dtype=float)
    for g, y in zip(got, ys):
        ref = float(phi_quad(fm, y))
        assert abs(g - ref) < 1e-15 * max(1.0, abs(ref)), (fam, y, g, ref)


@pytest.mark.parametrize("m,M", [(0, 16), (5, 64), (31, 64), (100, 256)])
def test_trapezoid_exact_on_transform_of_legendre(m, M):
    # feeding the exact phi of P_m through eq. (2.5) and the trapezoid form
    # of eq. (2.4) gives c_n = delta_{nm} for n < M/2 (no aliasing: n+m+1 < M)
    y = oracle.y_grid(M)
    phi = np.array([phi_legendre(m, float(abs(v))) for v in y], dtype=float).astype(LD)
    fh = oracle.fhat_from_phi(phi, y)
    c, imag = oracle.coeffs_from_fhat(fh, M // 2, return_imag=True)
    e = np.zeros(M // 2)
    e[m] = 1.0
    assert np.max(np.abs(np.array(c, dtype=float) - e)) < 1e-14
    assert imag < 1e-16


def test_fhat_symmetry_eq_2_12():
    # eq. (2.12): fhat(y) = -e^{iy} fhat(-y)
    f = W.Exponential(1.3)
    y = np.linspace(0.1, 3.0, 7, dtype=LD)
    a = oracle.abel_fhat(f, y, 24)
    b = oracle.abel_fhat(f, -y, 24)
    rhs = -np.exp(1j * y.astype(float)) * b.astype(complex)
    assert np.max(np.abs(a.astype(complex) - rhs)) < 1e-15


@pytest.mark.parametrize("D,N", [(20, 16), (63, 64)])
def test_method_exact_for_resolved_polynomial(D, N):
    # degree-D polynomial: Abel rule exact when 2Q-1 >= D, trapezoid exact
    # when M >= N + D + 1; then the method returns the true coefficients
    coef = np.random.default_rng(D).standard_normal(D + 1)
    f = W.LegendreSeries(coef)
    Q = (D + 1) // 2 + 1
    M = N + D + 1 + ((N + D + 1) % 2)
    c = np.array(oracle.method_coeffs(f, N, M, Q), dtype=float)
    assert np.max(np.abs(c - coef[:N])) < 5e-14


@pytest.mark.parametrize("M", [128, 160, 200])
def test_method_aliasing_law(M):
    # with phi resolved, the M-point grid returns
    #   a~_n = sum_{l>=0} a_{n+lM} - sum_{l>=1} a_{lM-1-n},  a_k = c_k/(2k+1)
    D, N = 100, 64
    coef = np.random.default_rng(7).standard_normal(D + 1)
    f = W.LegendreSeries(coef)
    c = np.array(oracle.method_coeffs(f, N, M, Q=52), dtype=float)
    a = coef / (2 * np.arange(D + 1) + 1)
    ak = lambda k: a[k] if 0 <= k <= D else 0.0
    for n in range(N):
        at = sum(ak(n + l * M) for l in range(0, 4)) - sum(ak(l * M - 1 - n) for l in range(1, 4))
        assert abs(c[n] - (2 * n + 1) * at) < 5e-13, (M, n)


def test_method_antisymmetric_discrete_spectrum():
    # a~_{M-1-n} = -a~_n for the full discrete spectrum
    M = 96
    f = W.GeneratingFunction(0.7)
    c = np.array(oracle.method_coeffs(f, M, M, 40), dtype=float)
    a = c / (2 * np.arange(M) + 1)
    assert np.max(np.abs(a + a[::-1])) < 1e-15


def test_method_small_workload_matches_definition():
    # N=64, M=256, Q=32: generating function t=0.5 and e^x
    for wl in W.single_small():
        cm = np.array(oracle.method_coeffs(wl.f, wl.N, wl.M, wl.Q), dtype=float)
        cd = np.array(oracle.legendre_coeffs(wl.f, wl.N, 128), dtype=float)
        assert np.max(np.abs(cm - cd)) < 1e-15 * np.max(np.abs(cd)), wl.name


def test_planted_twist_sign_is_caught():
    # dropping eps(y) (or the e^{iy/2}) in eq. (2.5) breaks the pin above
    M, m = 64, 5
    y = oracle.y_grid(M)
    phi = np.array([phi_legendre(m, float(abs(v))) for v in y], dtype=float).astype(LD)
    bad = oracle.fhat_from_phi(phi, np.abs(y))  # eps(y) lost
    c = np.array(oracle.coeffs_from_fhat(bad, M // 2), dtype=float)
    e = np.zeros(M // 2)
    e[m] = 1.0
    assert np.max(np.abs(c - e)) > 0.1


# ---------------------------------------------------------------------------
# The subset transform (eq. (2.4) evaluated only at listed indices n) and the
# sample builder of the [M/2][Q] layout.  Both feed full-size GPU parity
# tests, so each is pinned to closed forms, not only to the full transform.

@pytest.mark.parametrize("m,M", [(0, 16), (7, 64), (40, 256)])
def test_subset_transform_of_legendre_is_delta(m, M):
    # exact phi of P_m through eq. (2.5), then the trapezoid form of eq. (2.4)
    # at listed indices only: c_n = delta_{nm} (no aliasing for n + m + 1 < M)
    y = oracle.y_grid(M)
    phi = np.array([phi_legendre(m, float(abs(v))) for v in y], dtype=float).astype(LD)
    fh = oracle.fhat_from_phi(phi, y)
    H = M // 2
    idx = np.array(sorted({0, 1, m, max(0, m - 1), m + 1, H - 2, H - 1}), dtype=np.int64)
    a = oracle.fourier_coeffs_at(fh, idx)
    c = np.array((2 * idx.astype(LD) + 1) * a.real, dtype=float)
    assert np.max(np.abs(c - (idx == m))) < 1e-14
    assert float(np.max(np.abs(a.imag))) < 1e-16


def test_subset_transform_equals_full_transform():
    # the subset sum at indices 0, N-1 and both parities equals the full sum
    M, N = 200, 100
    f = W.Exponential(-2.5)
    fh = oracle.abel_fhat(f, oracle.y_grid(M), 24)
    full = oracle.fourier_coeffs(fh, N)
    idx = np.array([0, 1, 2, 37, 50, 98, N - 1], dtype=np.int64)
    sub = oracle.fourier_coeffs_at(fh, idx)
    assert np.max(np.abs(np.asarray(sub - full[idx], dtype=complex))) <= 1e-18


def test_method_coeffs_at_generating_function_closed_form():
    # t = 0.6 resolved by (M, Q): c_n = t^n (eq. (2.2)) at sampled indices
    t, M, Q = 0.6, 512, 48
    idx = np.array([0, 1, 2, 3, 10, 21, 40, 63, 255], dtype=np.int64)
    got = np.array(oracle.method_coeffs_at(W.GeneratingFunction(t), idx, M, Q), dtype=float)
    assert np.max(np.abs(got - t ** idx.astype(float))) < 5e-16
    full = oracle.method_coeffs(W.GeneratingFunction(t), 256, M, Q)
    assert np.max(np.abs(np.asarray(oracle.method_coeffs_at(W.GeneratingFunction(t), idx, M, Q)
                                    - full[idx], dtype=float))) <= 1e-18


def test_positive_half_samples_layout():
    # f(x) = x returns the nodes themselves: row j-1 holds y = pi j / H,
    # column q the q-th largest positive node T_q of the 2Q-point
    # Gauss-Legendre rule (numpy's leggauss here, an independent routine),
    # x = cos y + (1 - cos y) T_q^2 rounded to FP64
    M, Q = 40, 6
    H = M // 2
    s = oracle.positive_half_samples(lambda x: x, M, Q)
    assert s.shape == (H, Q) and s.dtype == np.float64
    T = np.sort(npleg.leggauss(2 * Q)[0])[::-1][:Q]
    y = np.pi * np.arange(1, H + 1) / H
    ref = np.cos(y)[:, None] + (1 - np.cos(y))[:, None] * T[None, :] ** 2
    assert np.max(np.abs(s - ref)) < 4e-16


@pytest.mark.parametrize("D,N", [(21, 16), (40, 32)])
def test_positive_half_samples_exact_polynomial(D, N):
    # samples of a degree-D series through the folded rule (2Q-1 >= D) and
    # the trapezoid (M >= N + D + 1) return its own coefficients
    coef = np.random.default_rng(100 + D).standard_normal(D + 1)
    f = W.LegendreSeries(coef)
    Q = (D + 1) // 2 + 1
    M = N + D + 2 + ((N + D) % 2)
    s = oracle.positive_half_samples(f, M, Q)
    c = np.array(oracle.method_coeffs_from_samples(s, N, M, Q), dtype=float)
    assert np.max(np.abs(c - coef[:N])) < 2e-14


def test_positive_half_samples_match_method_fp64_nodes():
    # the samples path equals the method with FP64-rounded nodes
    M, Q, N = 256, 20, 100
    f = W.Sum(W.GeneratingFunction(0.8), W.Exponential(3.0))
    s = oracle.positive_half_samples(f, M, Q)
    a = np.array(oracle.method_coeffs_from_samples(s, N, M, Q), dtype=float)
    b = np.array(oracle.method_coeffs(f, N, M, Q, fp64_nodes=True), dtype=float)
    assert np.max(np.abs(a - b)) < 1e-15 * np.max(np.abs(b))
