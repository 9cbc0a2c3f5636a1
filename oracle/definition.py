"""The definition of the Legendre coefficients, computed by brute force.

Test infrastructure only (see the package docstring).

Follows Section 2 of De Micheli & Viano (arXiv 1106.0463):

* eq. (2.1)  f(x) = sum_n c_n P_n(x) on [-1, 1];
* eq. (2.3)  c_n = (n + 1/2) * integral_{-1}^{1} f(x) P_n(x) dx.

The integral is evaluated with a K-point Gauss-Legendre rule built here by
Newton iteration in long double, and P_n(x_k) by the three-term recurrence.
This is the O(N K) "standard quadrature" route that the paper's
introduction contrasts with its own method.  It is exact (up to rounding)
whenever f P_n is a polynomial of degree <= 2K - 1, and converges
geometrically for f analytic on [-1, 1].
"""
from __future__ import annotations

import numpy as np

from . import _lib

LD = np.longdouble


def _ptr(a: np.ndarray):
    return a.ctypes.data


def gauss_legendre(K: int) -> tuple[np.ndarray, np.ndarray]:
    """Nodes (decreasing) and weights of the K-point Gauss-Legendre rule on
    [-1, 1], in long double."""
    K = int(K)
    if K < 1:
        raise ValueError("K must be >= 1")
    x = np.empty(K, dtype=LD)
    w = np.empty(K, dtype=LD)
    rc = _lib.load().oracle_gauss_legendre(K, _ptr(x), _ptr(w))
    if rc != 0:
        raise RuntimeError(f"oracle_gauss_legendre failed (rc={rc}, K={K})")
    return x, w


def legendre_coeffs_from_samples(x: np.ndarray, w: np.ndarray, fx: np.ndarray,
                                 N: int) -> np.ndarray:
    """c_n = (n+1/2) sum_k w_k f(x_k) P_n(x_k), n < N   (eq. 2.3 by quadrature)."""
    x = np.ascontiguousarray(x, dtype=LD)
    w = np.ascontiguousarray(w, dtype=LD)
    fx = np.ascontiguousarray(fx, dtype=LD)
    if not (x.shape == w.shape == fx.shape) or x.ndim != 1:
        raise ValueError("x, w, f(x) must be 1-D arrays of one length")
    c = np.empty(int(N), dtype=LD)
    rc = _lib.load().oracle_legendre_coeffs(x.size, _ptr(x), _ptr(w), _ptr(fx),
                                            int(N), _ptr(c))
    if rc != 0:
        raise RuntimeError(f"oracle_legendre_coeffs failed (rc={rc})")
    return c


def legendre_coeffs(f, N: int, K: int) -> np.ndarray:
    """First N Legendre coefficients of f (a callable on long-double arrays),
    eq. (2.3), with a K-point Gauss-Legendre rule.

    K must make f P_{N-1} integrable to the wanted accuracy: for a polynomial
    f of degree D, K >= (N + D) / 2 is exact.
    """
    x, w = gauss_legendre(K)
    fx = np.asarray(f(x), dtype=LD)
    return legendre_coeffs_from_samples(x, w, fx, N)


def legendre_coeffs_piecewise(f, N: int, K: int, breakpoints=()) -> np.ndarray:
    """eq. (2.3) with the K-point rule applied on each piece of [-1, 1] cut at
    ``breakpoints`` (for f smooth only piecewise, e.g. |x|^{3/2} at x = 0)."""
    cuts = [LD(-1)] + [LD(b) for b in sorted(breakpoints)] + [LD(1)]
    t, wt = gauss_legendre(K)
    xs, ws = [], []
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        half = (hi - lo) / 2
        mid = (hi + lo) / 2
        xs.append(mid + half * t)
        ws.append(half * wt)
    x = np.concatenate(xs)
    w = np.concatenate(ws)
    fx = np.asarray(f(x), dtype=LD)
    return legendre_coeffs_from_samples(x, w, fx, N)


def legendre_eval(c: np.ndarray, x: np.ndarray) -> np.ndarray:
    """sum_n c_n P_n(x), eq. (2.1) truncated, by the forward recurrence
    (used to check that the coefficients reconstruct f)."""
    x = np.asarray(x, dtype=LD)
    c = np.asarray(c, dtype=LD)
    p0 = np.ones_like(x)
    out = c[0] * p0
    if c.size == 1:
        return out
    p1 = x.copy()
    out = out + c[1] * p1
    for n in range(1, c.size - 1):
        p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1)
        out = out + c[n + 1] * p2
        p0, p1 = p1, p2
    return out
