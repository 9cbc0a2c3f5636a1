"""Closed-form Legendre coefficients and Abel transforms used to pin the
oracle (all computed with mpmath at high precision, independently of the
oracle's own quadrature and recurrences).

References are to De Micheli & Viano, arXiv 1106.0463, Section 2.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath as mp
import numpy as np

mp.mp.dps = 40


def genfn_coeffs(t: float, N: int) -> np.ndarray:
    """Generating function eq. (2.2): (1-2xt+t^2)^{-1/2} = sum P_n t^n,
    hence c_n = t^n."""
    return np.array([mp.mpf(t) ** n for n in range(N)], dtype=object)


def exp_coeffs(a: float, N: int) -> np.ndarray:
    """e^{a x} = sum_n (2n+1) i_n(a) P_n(x), with the modified spherical
    Bessel function i_n(z) = sqrt(pi/(2z)) I_{n+1/2}(z) and i_n(-z) =
    (-1)^n i_n(z); a = 0 gives delta_{n0}."""
    a = mp.mpf(a)
    out = []
    for n in range(N):
        if a == 0:
            out.append(mp.mpf(1) if n == 0 else mp.mpf(0))
            continue
        z = abs(a)
        i_n = mp.sqrt(mp.pi / (2 * z)) * mp.besseli(n + mp.mpf(1) / 2, z)
        sgn = 1 if (a > 0 or n % 2 == 0) else -1
        out.append((2 * n + 1) * sgn * i_n)
    return np.array(out, dtype=object)


def cos_coeffs(omega: float, N: int) -> np.ndarray:
    """cos(omega x) = sum_{n even} (2n+1) (-1)^{n/2} j_n(omega) P_n(x),
    j_n(z) = sqrt(pi/(2z)) J_{n+1/2}(z)."""
    w = mp.mpf(omega)
    out = []
    for n in range(N):
        if n % 2:
            out.append(mp.mpf(0))
            continue
        j_n = mp.sqrt(mp.pi / (2 * w)) * mp.besselj(n + mp.mpf(1) / 2, w)
        out.append((2 * n + 1) * (-1) ** (n // 2) * j_n)
    return np.array(out, dtype=object)


def cos_coeff(omega: float, n: int) -> mp.mpf:
    """One coefficient of :func:`cos_coeffs`."""
    if n % 2:
        return mp.mpf(0)
    w = mp.mpf(omega)
    return (2 * n + 1) * (-1) ** (n // 2) * mp.sqrt(mp.pi / (2 * w)) * mp.besselj(n + mp.mpf(1) / 2, w)


def abs_pow_coeffs(N: int, alpha: Fraction = Fraction(3, 2)) -> list:
    """Closed form printed before Table 1 (Section 2) for f = |x|^alpha,
    read as: 0 for odd n; 1/(alpha+1) for n = 0; otherwise
    (2n+1) prod_{k=0}^{n/2-1} (alpha - 2k) / prod_{k=0}^{n/2} (alpha + 1 + 2k).
    Exact rationals."""
    out = []
    for n in range(N):
        if n % 2:
            out.append(Fraction(0))
        elif n == 0:
            out.append(1 / (alpha + 1))
        else:
            num = Fraction(2 * n + 1)
            for k in range(n // 2):
                num *= alpha - 2 * k
            den = Fraction(1)
            for k in range(n // 2 + 1):
                den *= alpha + 1 + 2 * k
            out.append(num / den)
    return out


def phi_legendre(m: int, y) -> float:
    """phi(y) of eq. (2.14) for f = P_m: 2 sin((m+1/2) y) / (2m+1).
    (It is pinned separately against mpmath quadrature of eq. (2.14).)"""
    return 2 * mp.sin((m + mp.mpf(1) / 2) * mp.mpf(y)) / (2 * m + 1)


def phi_quad(f_mp, y) -> mp.mpf:
    """phi(y) of eq. (2.14), integral_{cos y}^1 f(x)/sqrt(2(x - cos y)) dx,
    by mpmath's tanh-sinh quadrature (handles the end-point singularity)."""
    y = mp.mpf(y)
    cy = mp.cos(y)
    return mp.quad(lambda x: f_mp(x) / mp.sqrt(2 * (x - cy)), [cy, 1])


def coeff_quad(f_mp, n: int, breakpoints=()) -> mp.mpf:
    """c_n of eq. (2.3) by mpmath's adaptive quadrature."""
    pts = [-1] + list(breakpoints) + [1]
    return (n + mp.mpf(1) / 2) * mp.quad(lambda x: f_mp(x) * mp.legendre(n, x), pts)


def load_table1(path: str) -> tuple[list[int], list[str]]:
    ns, vals = [], []
    with open(path) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            a, b = line.split()
            ns.append(int(a))
            vals.append(b)
    return ns, vals


def phi_genfn(t: float, y) -> mp.mpf:
    """phi(y) of eq. (2.14) for the generating function eq. (2.2),
    (1 - 2xt + t^2)^{-1/2}: since its c_n = t^n and phi_{P_n} =
    2 sin((n+1/2) y)/(2n+1), phi = sum_n t^n 2 sin((n+1/2) y)/(2n+1)
    = Im[(2/sqrt(t)) artanh(sqrt(t) e^{iy/2})]."""
    t, y = mp.mpf(t), mp.mpf(y)
    z = mp.sqrt(t) * mp.exp(1j * y / 2)
    return mp.im(2 / mp.sqrt(t) * mp.atanh(z))


def phi_cos(omega: float, y) -> mp.mpf:
    """phi(y) of eq. (2.14) for f = cos(omega x): with x = cos y + u^2/2,
    phi = integral_0^{2 sin(y/2)} cos(omega (cos y + u^2/2)) du
        = sqrt(pi/omega) [cos(omega cos y) C(z) - sin(omega cos y) S(z)],
    z = 2 sin(y/2) sqrt(omega/pi), C and S the Fresnel integrals."""
    w, y = mp.mpf(omega), mp.mpf(y)
    z = 2 * mp.sin(y / 2) * mp.sqrt(w / mp.pi)
    cy = mp.cos(y)
    return mp.sqrt(mp.pi / w) * (mp.cos(w * cy) * mp.fresnelc(z) - mp.sin(w * cy) * mp.fresnels(z))


def exp_coeffs_fast(a: float, N: int) -> np.ndarray:
    """The coefficients of :func:`exp_coeffs` in float64 for large N:
    c_n = (2n+1) sgn(a)^n i_n(|a|), with i_n by Miller's backward
    recurrence i_{n-1}(z) = i_{n+1}(z) + (2n+1)/z i_n(z) (stable downward:
    i_n is the recurrence's minimal solution) in long double, normalised by
    i_0(z) = sinh(z)/z.  Values below the float64 range come out as 0; the
    start index lies 60 above the last index kept (at most 600: beyond it
    every c_n with |a| <= 40 is far below 1e-300)."""
    N = int(N)
    out = np.zeros(N, dtype=np.float64)
    if a == 0:
        out[0] = 1.0
        return out
    z = np.longdouble(abs(a))
    top = min(N - 1, 600)
    start = top + 60 + int(abs(a))
    vals = np.zeros(top + 1, dtype=np.longdouble)
    big = np.longdouble("1e4000")
    ip1, i = np.longdouble(0), np.longdouble("1e-4000")
    for n in range(start, 0, -1):
        im1 = ip1 + (2 * n + 1) / z * i
        if n - 1 <= top:
            vals[n - 1] = im1
        ip1, i = i, im1
        if i > big:                         # rescale (long double range)
            ip1 /= big
            i /= big
            vals /= big
    i0 = np.sinh(z) / z
    vals *= i0 / vals[0]
    n = np.arange(top + 1)
    sgn = np.where((a > 0) | (n % 2 == 0), 1.0, -1.0)
    out[:top + 1] = ((2 * n + 1) * vals).astype(np.float64) * sgn
    return out


def exp_coeffs_many(a, top: int = 600) -> np.ndarray:
    """:func:`exp_coeffs_fast` for many exponents at once: row k holds
    c_0..c_top of e^{a_k x} (|a_k| <= 40), the same backward recurrence run
    on all rows together in long double."""
    a = np.asarray(a, dtype=np.float64)
    z = np.abs(a).astype(np.longdouble)
    zs = np.where(z == 0, np.longdouble(1), z)
    big = np.longdouble("1e4000")
    start = top + 60 + 40
    vals = np.zeros((a.size, top + 1), dtype=np.longdouble)
    ip1 = np.zeros(a.size, dtype=np.longdouble)
    i = np.full(a.size, np.longdouble("1e-4000"))
    for n in range(start, 0, -1):
        im1 = ip1 + (2 * n + 1) / zs * i
        if n - 1 <= top:
            vals[:, n - 1] = im1
        ip1, i = i, im1
        hot = i > big
        if np.any(hot):
            ip1[hot] /= big
            i[hot] /= big
            vals[hot] /= big
    i0 = np.sinh(zs) / zs
    vals *= (i0 / vals[:, 0])[:, None]
    n = np.arange(top + 1)
    sgn = np.where((a[:, None] > 0) | (n[None, :] % 2 == 0), 1.0, -1.0)
    out = ((2 * n + 1)[None, :] * vals).astype(np.float64) * sgn
    out[z == 0] = 0.0
    out[z == 0, 0] = 1.0
    return out
