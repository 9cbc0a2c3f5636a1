"""The paper's discretized method, step by step, on the CPU.

Test infrastructure only (see the package docstring).

De Micheli & Viano (arXiv 1106.0463), Section 2:

1. Theorem 1, eq. (2.5): the Abel-type transform
       fhat(y) = (1 / (2 pi i)) eps(y) e^{i y/2} phi(|y|),
   with eq. (2.14)
       phi(y) = integral_{cos y}^{1} f(x) / sqrt(2 (x - cos y)) dx.
   The end-point singularity is removed by a nonlinear change of variable
   followed by Gauss-Legendre quadrature (the numerical remarks after
   eq. (2.14)).  The paper does not print the substitution; the reading used
   here is x = cos y + L t^2 with L = 1 - cos y, so that
       dx / sqrt(2 (x - cos y)) = sqrt(2 L) dt,
       phi(y) = sqrt(2 L) * integral_0^1 f(cos y + L t^2) dt,
   and, the integrand being even in t,
       integral_0^1 g(t) dt = (1/2) integral_{-1}^{1} g(t) dt,
   which is evaluated with the (2Q)-point Gauss-Legendre rule on [-1, 1].
2. Theorem 1, eq. (2.4): a_n = integral_{-pi}^{pi} fhat(y) e^{i n y} dy, by
   the trapezoid rule on the periodic grid y_j = -pi + 2 pi j / M (the
   discrete Fourier transform that the paper evaluates with one FFT; here it
   is a plain O(M N) sum).
3. Definition in Theorem 1: c_n = (2n + 1) a_n.

Everything is long double.  The result agrees with eq. (2.3) up to the two
discretization errors (Abel quadrature with Q, trapezoid with M).
"""
from __future__ import annotations

import numpy as np

from . import _lib
from .definition import gauss_legendre

LD = np.longdouble
PI = LD("3.141592653589793238462643383279502884")


def abel_nodes(y: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Abel nodes x = cos y + (1 - cos y) T^2 for each y (rows) and each
    Gauss node T (columns), long double."""
    y = np.asarray(y, dtype=LD)
    cy = np.cos(y)
    L = 1 - cy                              # length of [cos y, 1]
    return cy[:, None] + L[:, None] * (np.asarray(T, dtype=LD)[None, :] ** 2)


def abel_phi(f, y: np.ndarray, Q: int, chunk: int = 2048, fp64_nodes: bool = False) -> np.ndarray:
    """phi(y) of eq. (2.14) for y in [-pi, pi] (even in y), with the
    (2Q)-point Gauss-Legendre rule after x = cos y + (1 - cos y) t^2
    (evaluated in blocks of ``chunk`` y values to bound memory).

    fp64_nodes=True rounds every node to the nearest FP64 value before f is
    evaluated (in long double) there: the samples an FP64 caller provides.
    """
    y = np.asarray(y, dtype=LD)
    T, W = gauss_legendre(2 * int(Q))
    out = np.empty(y.shape, dtype=LD)
    for a in range(0, y.size, chunk):
        yy = y[a:a + chunk]
        x = abel_nodes(yy, T)
        if fp64_nodes:
            x = x.astype(np.float64).astype(LD)
        fx = np.asarray(f(x), dtype=LD)
        integral = LD(0.5) * (fx * W[None, :]).sum(axis=1)
        out[a:a + chunk] = np.sqrt(2 * (1 - np.cos(yy))) * integral
    return out


def fhat_from_phi(phi_abs_y: np.ndarray, y: np.ndarray) -> np.ndarray:
    """fhat(y) of eq. (2.5) given phi(|y|):
    (1/(2 pi i)) eps(y) e^{i y/2} phi(|y|)."""
    y = np.asarray(y, dtype=LD)
    eps = np.sign(y)
    # 1/(2 pi i) = -i/(2 pi);  e^{i y/2} = cos(y/2) + i sin(y/2)
    mag = eps * np.asarray(phi_abs_y, dtype=LD) / (2 * PI)
    return (-1j) * mag * (np.cos(y / 2) + 1j * np.sin(y / 2))


def abel_fhat(f, y: np.ndarray, Q: int, fp64_nodes: bool = False) -> np.ndarray:
    """fhat(y) of eq. (2.5) with phi from :func:`abel_phi`."""
    y = np.asarray(y, dtype=LD)
    return fhat_from_phi(abel_phi(f, np.abs(y), Q, fp64_nodes=fp64_nodes), y)


def fourier_coeffs(fhat_vals: np.ndarray, N: int) -> np.ndarray:
    """a_n = (2 pi / M) sum_j fhat(y_j) e^{i n y_j}, y_j = -pi + 2 pi j / M,
    n < N: the trapezoid rule for eq. (2.4).  Returns complex long double."""
    fh = np.asarray(fhat_vals)
    re = np.ascontiguousarray(fh.real, dtype=LD)
    im = np.ascontiguousarray(fh.imag, dtype=LD)
    M = re.size
    a_re = np.empty(int(N), dtype=LD)
    a_im = np.empty(int(N), dtype=LD)
    rc = _lib.load().oracle_fourier_coeffs(M, re.ctypes.data, im.ctypes.data,
                                           int(N), a_re.ctypes.data,
                                           a_im.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_fourier_coeffs failed (rc={rc})")
    return a_re + 1j * a_im


def fourier_coeffs_at(fhat_vals: np.ndarray, idx) -> np.ndarray:
    """:func:`fourier_coeffs` for the listed indices only."""
    fh = np.asarray(fhat_vals)
    re = np.ascontiguousarray(fh.real, dtype=LD)
    im = np.ascontiguousarray(fh.imag, dtype=LD)
    ii = np.ascontiguousarray(idx, dtype=np.int64)
    a_re = np.empty(ii.size, dtype=LD)
    a_im = np.empty(ii.size, dtype=LD)
    rc = _lib.load().oracle_fourier_coeffs_idx(re.size, re.ctypes.data, im.ctypes.data, ii.size,
                                               ii.ctypes.data, a_re.ctypes.data, a_im.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_fourier_coeffs_idx failed (rc={rc})")
    return a_re + 1j * a_im


def method_coeffs_at(f, idx, M: int, Q: int, fp64_nodes: bool = False) -> np.ndarray:
    """:func:`method_coeffs` evaluated only at the indices ``idx``."""
    y = y_grid(M)
    fh = abel_fhat(f, y, Q, fp64_nodes)
    a = fourier_coeffs_at(fh, idx)
    n = np.asarray(idx, dtype=LD)
    return (2 * n + 1) * a.real


def positive_half_samples(f, M: int, Q: int) -> np.ndarray:
    """Samples f(x) at the FP64-rounded Abel nodes of the positive half of
    the grid, y = pi j / (M/2), j = 1..M/2 (rows), and the positive Gauss
    nodes in decreasing order (columns): the [M/2][Q] layout an FP64 caller
    hands to a single-function execution.  Uses the same grid values and
    nodes as :func:`method_coeffs` with ``fp64_nodes=True``."""
    H = int(M) // 2
    yg = np.abs(y_grid(M))
    y = np.concatenate([yg[H + 1:], yg[:1]])   # pi j / H for j = 1..H-1, then pi
    T, _ = gauss_legendre(2 * int(Q))
    out = np.empty((H, int(Q)), dtype=np.float64)
    for a in range(0, H, 2048):
        x = abel_nodes(y[a:a + 2048], T[:int(Q)]).astype(np.float64).astype(LD)
        out[a:a + 2048] = np.asarray(f(x), dtype=LD).astype(np.float64)
    return out


def y_grid(M: int) -> np.ndarray:
    """The periodic trapezoid grid y_j = -pi + 2 pi j / M, j = 0..M-1."""
    j = np.arange(int(M), dtype=LD)
    return -PI + 2 * PI * j / LD(M)


def coeffs_from_fhat(fhat_vals: np.ndarray, N: int, return_imag: bool = False):
    """c_n = (2n+1) a_n with a_n from :func:`fourier_coeffs` (Theorem 1)."""
    a = fourier_coeffs(fhat_vals, N)
    n = np.arange(int(N), dtype=LD)
    c = (2 * n + 1) * a.real
    if return_imag:
        return c, np.max(np.abs(a.imag))
    return c


def method_coeffs(f, N: int, M: int, Q: int, return_imag: bool = False,
                  fp64_nodes: bool = False):
    """c_0..c_{N-1} by the paper's method with an M-point y-grid and the
    (2Q)-point Gauss-Legendre rule for the Abel integral.

    Steps in the paper's order: fhat on the grid (eq. 2.5 / 2.14), the
    Fourier coefficients a_n (eq. 2.4), c_n = (2n+1) a_n (Theorem 1).
    For real f the a_n are real; the largest imaginary part is returned on
    request as a consistency check.
    """
    y = y_grid(M)
    fh = abel_fhat(f, y, Q, fp64_nodes)
    return coeffs_from_fhat(fh, N, return_imag)
