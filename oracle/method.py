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


# ----------------------------------------------------------------------------
# Composite Abel rule (breakpoints, grading toward x = 1, per-row node counts)
#
# With x = 1 - 2 s^2 (1 - t^2), s = sin(y/2), the Abel integral eq. (2.14) is
#     phi(y) = 2 s * integral_0^1 f(1 - 2 s^2 (1 - t^2)) dt
# (the substitution of the paper's numerical remarks, as in abel_phi).  A
# composite rule cuts t in [0, 1] into panels:
#   * a breakpoint b of f with cos y < b < 1 (a point where f or one of its
#     derivatives jumps, e.g. x = 0 for |x|^{3/2}) becomes the cut
#     t_b = sqrt(1 - r) with r = (1 - b) / (2 s^2), i.e. 1 - t_b = r / (1 + sqrt(1 - r));
#   * grading toward t = 1 (x = 1), for f with a singularity just beyond
#     x = 1, adds the cuts 1 - t = sigma^k, k = 1..K.
# Cuts are handled by their distance e = 1 - t; cuts with e <= 1e-15 or
# e >= 1 - 1e-7 (t <= 1e-7: a breakpoint within ~1e-14 of cos y, the row's
# own end point) are dropped, and a cut closer than 1e-12 max(e) to the
# previous one (in decreasing e) is merged into it.
# The first panel [0, t_1] uses the positive half of the 2q-point
# Gauss-Legendre rule (the integrand is even in t there); every other panel
# uses the q-point rule.  The node count of a panel [t_lo, t_hi] is q, or,
# for f band-limited to degree ~D,
#     q_p = min(q_max, ladder(q + ceil(g))),  g = G + 6.5 G^{1/3},
#     G = (D s^2 / 2) (t_hi^2 - t_lo^2):
# cos(D x) needs about D s^2 / 2 nodes for the whole row (a law measured on
# its closed-form transform; a uniform rule needs D / 2 in every row), and
# the phase of cos(D (1 - 2 s^2 (1 - t^2))) is spread over t in proportion
# to t^2, so each panel gets its share.  ladder(n) rounds up to a multiple
# of 8 for n <= 128 and to a multiple of 2^(floor(log2 n) - 4) above (16
# steps per octave), so that a plan needs about a hundred distinct rules.

def abel_rule_row_q(s, rule: dict) -> int:
    """Node count of a whole row [0, 1] with s = sin(y/2) under ``rule``."""
    return abel_rule_panel_q(s, LD(0), LD(1), rule)


def abel_rule_panel_q(s, t_lo, t_hi, rule: dict) -> int:
    """Node count of the panel [t_lo, t_hi] of a row with s = sin(y/2)."""
    q = int(rule["q"])
    D = float(rule.get("band", 0.0))
    if D <= 0:
        return q
    g = LD(D) * LD(s) ** 2 / 2 * (LD(t_hi) ** 2 - LD(t_lo) ** 2)
    g = g + LD(6.5) * np.cbrt(g)
    qj = abel_rule_ladder(q + int(np.ceil(g)))
    return min(int(rule.get("q_max", qj)), qj)


def abel_rule_ladder(n: int) -> int:
    """Smallest ladder value >= n: multiples of 8 up to 128, then multiples
    of 2^(floor(log2 n) - 4)."""
    n = int(n)
    if n <= 128:
        return 8 * ((n + 7) // 8)
    step = 1 << (n.bit_length() - 1 - 4)
    return step * ((n + step - 1) // step)


def abel_rule_cuts(s, rule: dict) -> list:
    """Cut distances e = 1 - t in (0, 1), decreasing, for one row."""
    s = LD(s)
    c = 1 - 2 * s * s                                   # cos y
    es = []
    for b in rule.get("breaks", ()):
        b = LD(b)
        if c < b < 1:
            r = (1 - b) / (2 * s * s)
            es.append(r / (1 + np.sqrt(1 - r)))
    sigma = float(rule.get("grade_ratio", 0.0))
    for k in range(1, int(rule.get("grade_levels", 0)) + 1):
        if sigma > 0:
            es.append(LD(sigma) ** k)
    es = sorted((e for e in es if LD(1e-15) < e < 1 - LD(1e-7)), reverse=True)
    out = []
    for e in es:
        if out and out[-1] - e < LD(1e-12) * out[0]:
            continue
        out.append(e)
    return out


def _half_rule(q: int):
    T, W = gauss_legendre(2 * q)
    return T[:q], W[:q]                                  # positive half, decreasing


def abel_phi_rule(f, y: np.ndarray, rule: dict, fp64_nodes: bool = False) -> np.ndarray:
    """phi(y) of eq. (2.14) for y in (0, pi] by the composite rule above.
    fp64_nodes=True rounds the nodes to FP64 before f is evaluated (the
    samples an FP64 caller provides)."""
    y = np.asarray(y, dtype=LD)
    out = np.empty(y.shape, dtype=LD)
    rules = {}
    for i, yy in enumerate(y.ravel()):
        s = np.sin(yy / 2)
        if s == 0:
            out.ravel()[i] = 0
            continue
        cuts = abel_rule_cuts(s, rule)
        bounds = [LD(1)] + cuts + [LD(0)]                # e = 1 - t at panel ends
        e_list, w_list = [], []
        # first panel [0, t_1]: t = t_1 T, 1 - t = e_1 + t_1 (1 - T)
        e1 = bounds[1]
        t1 = 1 - e1
        q = abel_rule_panel_q(s, LD(0), t1, rule)
        if ("h", q) not in rules:
            rules[("h", q)] = _half_rule(q)
        T, W = rules[("h", q)]
        e_list.append(e1 + t1 * (1 - T))
        w_list.append(t1 * W)
        # panels [t_p, t_{p+1}]: 1 - t = e_{p+1} + h (1 - tau), h = (e_p - e_{p+1}) / 2
        for p in range(1, len(bounds) - 1):
            q = abel_rule_panel_q(s, 1 - bounds[p], 1 - bounds[p + 1], rule)
            if ("f", q) not in rules:
                rules[("f", q)] = gauss_legendre(q)
            tau, om = rules[("f", q)]
            h = (bounds[p] - bounds[p + 1]) / 2
            e_list.append(bounds[p + 1] + h * (1 - tau))
            w_list.append(h * om)
        e = np.concatenate(e_list)
        w = np.concatenate(w_list)
        x = 1 - 2 * s * s * (e * (2 - e))
        if fp64_nodes:
            x = x.astype(np.float64).astype(LD)
        out.ravel()[i] = 2 * s * np.sum(w * np.asarray(f(x), dtype=LD))
    return out


def abel_rule_node_count(M: int, rule: dict) -> int:
    """Number of Abel nodes of the composite rule over y = pi j / (M/2),
    j = 1..M/2."""
    H = int(M) // 2
    n = 0
    for j in range(1, H + 1):
        s = np.sin(PI * j / (2 * H))
        bounds = [LD(1)] + abel_rule_cuts(s, rule) + [LD(0)]
        for p in range(len(bounds) - 1):
            t_lo = LD(0) if p == 0 else 1 - bounds[p]
            n += abel_rule_panel_q(s, t_lo, 1 - bounds[p + 1], rule)
    return n


def method_coeffs_rule(f, N: int, M: int, rule: dict, fp64_nodes: bool = False) -> np.ndarray:
    """c_0..c_{N-1} by the method with the composite Abel rule: phi on the
    positive half of the M-point grid, then eq. (2.5), the trapezoid form of
    eq. (2.4) and c_n = (2n+1) a_n, as in :func:`method_coeffs`."""
    y = y_grid(M)
    H = int(M) // 2
    j = np.arange(1, H + 1, dtype=LD)
    yp = PI * j / H                                       # the distinct |y| > 0
    phi_pos = abel_phi_rule(f, yp, rule, fp64_nodes)
    # |y_k| = pi |k - H| / H on the grid y_k = -pi + 2 pi k / M
    k = np.arange(int(M))
    idx = np.abs(k - H)
    phi_abs = np.where(idx == 0, LD(0), phi_pos[np.maximum(idx, 1) - 1])
    fh = fhat_from_phi(phi_abs, y)
    return coeffs_from_fhat(fh, N)


# ----------------------------------------------------------------------------
# Two-dimensional tensor-product transform (the extension named in the
# paper's closing remarks):
#     c_{nm} = (n + 1/2)(m + 1/2) integral integral f(x1, x2) P_n(x1) P_m(x2),
# by the one-dimensional method along x1 for every sample point of x2, then
# along x2 for every n.  Both axes use the same Abel nodes (the positive half
# of the grid times the Gauss nodes), so the samples are f(X_a, X_b) on the
# product of the 1-D node set with itself.

def abel_node_set(M: int, Q: int) -> np.ndarray:
    """The 1-D Abel nodes in the [M/2][Q] layout of positive_half_samples
    (rows y = pi j / (M/2), j = 1..M/2; columns the positive Gauss nodes,
    decreasing), long double."""
    H = int(M) // 2
    yg = np.abs(y_grid(M))
    y = np.concatenate([yg[H + 1:], yg[:1]])
    T, _ = gauss_legendre(2 * int(Q))
    return abel_nodes(y, T[:int(Q)])


def method_coeffs_from_samples(samples: np.ndarray, N: int, M: int, Q: int) -> np.ndarray:
    """The method from given samples s[j-1][q] = f(x_{jq}) at the nodes of
    :func:`abel_node_set` (the last axis may carry several functions:
    s[j-1][q][k]): phi_j = 2 sin(y_j/2) (1/2) sum_q W_q s[j][q] (the folded
    2Q-point rule of abel_phi), then eq. (2.5), the trapezoid form of
    eq. (2.4) and c_n = (2n+1) a_n.  Returns [N] or [N][k]."""
    s = np.asarray(samples, dtype=LD)
    H = int(M) // 2
    T, W = gauss_legendre(2 * int(Q))
    # the full 2Q-point sum of an even integrand is twice the positive half
    integral = LD(0.5) * 2 * np.tensordot(W[:int(Q)], s, axes=([0], [1]))   # [H] or [H][k]
    j = np.arange(1, H + 1, dtype=LD)
    yp = PI * j / H
    phi_pos = (np.sqrt(2 * (1 - np.cos(yp))) * integral.T).T
    y = y_grid(M)
    k = np.arange(int(M))
    idx = np.abs(k - H)
    sel = np.maximum(idx, 1) - 1
    phi_abs = phi_pos[sel]
    phi_abs[idx == 0] = 0
    if phi_abs.ndim == 1:
        return coeffs_from_fhat(fhat_from_phi(phi_abs, y), N)
    out = np.empty((int(N), phi_abs.shape[1]), dtype=LD)
    for c in range(phi_abs.shape[1]):
        out[:, c] = coeffs_from_fhat(fhat_from_phi(phi_abs[:, c], y), N)
    return out


def method_coeffs_2d(f2, N: int, M: int, Q: int, fp64_nodes: bool = True) -> np.ndarray:
    """c[n1][n2] of f2(x1, x2) by the method along x1 (for every node of x2),
    then along x2.  fp64_nodes rounds the nodes to FP64 before f2 is
    evaluated (long double) there."""
    X = abel_node_set(M, Q).reshape(-1)
    if fp64_nodes:
        X = X.astype(np.float64).astype(LD)
    H, Qi = int(M) // 2, int(Q)
    F = np.asarray(f2(X[:, None], X[None, :]), dtype=LD)          # F[a][b] = f(X_a, X_b)
    c1 = method_coeffs_from_samples(F.reshape(H, Qi, -1), N, M, Q)   # [n1][b]
    c2 = method_coeffs_from_samples(c1.T.reshape(H, Qi, -1), N, M, Q)  # [n2][n1]
    return c2.T
