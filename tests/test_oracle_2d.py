"""Pins of the oracle's two-dimensional tensor-product transform (the 1-D
method along x1, then along x2) against the mathematics: Legendre products
P_a(x1) P_b(x2) give one unit coefficient, a separable product gives the
outer product of closed-form 1-D coefficients, and a non-separable f agrees
with eq. (2.3) applied along both axes by Gauss-Legendre quadrature."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
import workloads as W
from closed_forms import exp_coeffs

LD = np.longdouble


def test_from_samples_matches_method():
    f = W.Exponential(0.7)
    N, M, Q = 16, 64, 8
    X = oracle.abel_node_set(M, Q).astype(np.float64).astype(LD)
    a = oracle.method_coeffs_from_samples(f(X), N, M, Q)
    b = oracle.method_coeffs(f, N, M, Q, fp64_nodes=True)
    assert np.max(np.abs(np.asarray(a - b, dtype=float))) < 1e-17


@pytest.mark.parametrize("a,b", [(0, 0), (3, 0), (2, 5), (7, 7)])
def test_legendre_products(a, b):
    # exact when the Abel rule and the grid resolve degree max(a, b)
    N, M, Q = 12, 48, 8
    ca = np.zeros(a + 1); ca[a] = 1
    cb = np.zeros(b + 1); cb[b] = 1
    f2 = lambda x1, x2: (npleg.legval(np.asarray(x1, dtype=np.float64), ca) *
                         npleg.legval(np.asarray(x2, dtype=np.float64), cb))
    C = np.asarray(oracle.method_coeffs_2d(f2, N, M, Q), dtype=float)
    E = np.zeros((N, N)); E[a, b] = 1
    assert np.max(np.abs(C - E)) < 1e-14


def test_separable_product_closed_forms():
    N, M, Q = 20, 128, 24
    t = 0.4
    f2 = lambda x1, x2: np.exp(LD(0.9) * x1) * W.GeneratingFunction(t)(x2)
    C = np.asarray(oracle.method_coeffs_2d(f2, N, M, Q), dtype=float)
    c1 = np.array([float(v) for v in exp_coeffs(0.9, N)])
    c2 = t ** np.arange(N)
    assert np.max(np.abs(C - np.outer(c1, c2))) < 1e-13


def test_nonseparable_against_definition():
    # f = exp(x1 x2): eq. (2.3) along both axes with a K-point rule per axis
    N, M, Q, K = 16, 96, 20, 40
    f2 = lambda x1, x2: np.exp(x1 * x2)
    C = np.asarray(oracle.method_coeffs_2d(f2, N, M, Q), dtype=float)
    x, w = oracle.gauss_legendre(K)
    F = np.exp(x[:, None] * x[None, :])
    step = np.stack([oracle.legendre_coeffs_from_samples(x, w, F[:, k], N) for k in range(K)], axis=1)
    D = np.stack([oracle.legendre_coeffs_from_samples(x, w, step[n, :], N) for n in range(N)], axis=0)
    assert np.max(np.abs(C - np.asarray(D, dtype=float))) < 1e-13
