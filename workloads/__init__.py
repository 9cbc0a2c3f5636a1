"""Seeded synthetic inputs for the Legendre-coefficient method.

This module is shared by the CPU oracle's tests and by the GPU tests and
benchmark, and for that reason holds none of the method's arithmetic: only
test functions f(x) (evaluated with numpy on float64 or long-double arrays,
or with torch on device tensors) and the seeded recipes that draw their
parameters.

Function families (the ones the paper names for its tests, Section 2, and
the generating function of eq. (2.2)):

* :class:`GeneratingFunction`  (1 - 2 x t + t^2)^{-1/2}, coefficients t^n
* :class:`Exponential`         e^{a x}
* :class:`Cosine`              cos(omega x)
* :class:`AbsPower`            |x|^alpha   (Table 1 uses alpha = 3/2)
* :class:`Rational`            (1 + x) / (gamma^2 + x^2)
* :class:`LegendreSeries`      sum_n c_n P_n(x) by Clenshaw's recurrence
* :class:`Sum`                 f + g
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _scalar_like(x, v):
    """v as a scalar of x's floating dtype (numpy) or a python float."""
    if isinstance(x, np.ndarray):
        return x.dtype.type(v)
    return v


@dataclass
class GeneratingFunction:
    """f(x) = (1 - 2 x t + t^2)^{-1/2}, written as ((1-t)^2 + 2t(1-x))^{-1/2}
    (the same value, without cancellation for t, x near 1)."""
    t: float
    name: str = "genfn"

    def __call__(self, x):
        t = _scalar_like(x, self.t)
        one = _scalar_like(x, 1.0)
        return one / np.sqrt((one - t) ** 2 + 2 * t * (one - x))

    def torch(self, x):
        import torch
        t = float(self.t)
        return torch.rsqrt((1.0 - t) ** 2 + (2.0 * t) * (1.0 - x))

    def torch_omx(self, omx):
        """The same from the complement 1 - x of the node (accurate near
        x = 1, where f is steep for t near 1)."""
        import torch
        t = float(self.t)
        return torch.rsqrt((1.0 - t) ** 2 + (2.0 * t) * omx)


@dataclass
class Exponential:
    """f(x) = e^{a x}."""
    a: float
    name: str = "exp"

    def __call__(self, x):
        return np.exp(_scalar_like(x, self.a) * x)

    def torch(self, x):
        import torch
        return torch.exp(float(self.a) * x)


@dataclass
class Cosine:
    """f(x) = cos(omega x)."""
    omega: float
    name: str = "cos"

    def __call__(self, x):
        return np.cos(_scalar_like(x, self.omega) * x)

    def torch(self, x):
        import torch
        return torch.cos(float(self.omega) * x)


@dataclass
class AbsPower:
    """f(x) = |x|^alpha."""
    alpha: float = 1.5
    name: str = "abspow"

    def __call__(self, x):
        return np.abs(x) ** _scalar_like(x, self.alpha)

    def torch(self, x):
        import torch
        return torch.abs(x) ** float(self.alpha)


@dataclass
class Rational:
    """f(x) = (1 + x) / (gamma^2 + x^2)."""
    gamma: float
    name: str = "rational"

    def __call__(self, x):
        g = _scalar_like(x, self.gamma)
        return (1 + x) / (g * g + x * x)

    def torch(self, x):
        g = float(self.gamma)
        return (1.0 + x) / (g * g + x * x)


@dataclass
class LegendreSeries:
    """f(x) = sum_{n<len(c)} c_n P_n(x), evaluated with Clenshaw's backward
    recurrence b_k = c_k + (2k+1)/(k+1) x b_{k+1} - (k+1)/(k+2) b_{k+2},
    f = b_0."""
    coeffs: np.ndarray
    name: str = "series"

    def __call__(self, x):
        x = np.asarray(x)
        dt = x.dtype if x.dtype in (np.float64, np.longdouble) else np.dtype(np.float64)
        x = x.astype(dt, copy=False)
        c = np.asarray(self.coeffs, dtype=dt)
        one = dt.type(1)
        b1 = np.zeros_like(x)
        b2 = np.zeros_like(x)
        for k in range(c.size - 1, -1, -1):
            alpha = dt.type(2 * k + 1) / dt.type(k + 1)
            beta = dt.type(k + 1) / dt.type(k + 2)
            b0 = c[k] + alpha * x * b1 - beta * b2
            b2, b1 = b1, b0
        return b1 * one

    @property
    def degree(self) -> int:
        return int(np.asarray(self.coeffs).size) - 1


@dataclass
class Sum:
    """f = g + h."""
    g: object
    h: object
    name: str = "sum"

    def __call__(self, x):
        return self.g(x) + self.h(x)

    def torch(self, x):
        return self.g.torch(x) + self.h.torch(x)


# --------------------------------------------------------------------------
# Seeded workload recipes.  Seeds are the workload's number (1..5); draws are
# made in the order written below.
# --------------------------------------------------------------------------

@dataclass
class SingleWorkload:
    """One function, N coefficients, an M-point y-grid, Q Abel nodes."""
    name: str
    f: object
    N: int
    M: int
    Q: int
    extra: dict = field(default_factory=dict)


def single_small() -> list[SingleWorkload]:
    """Small single-function workload: N=64, M=256, Q=32, FP64, for
    f = (1 - x + 0.25)^{-1/2} (t = 0.5, c_n = 0.5^n) and f = e^x."""
    return [SingleWorkload("genfn_t0.5", GeneratingFunction(0.5), 64, 256, 32),
            SingleWorkload("exp_a1", Exponential(1.0), 64, 256, 32)]


def single_large(Q: int = 64) -> SingleWorkload:
    """Large oscillatory single function: f = cos(omega x) +
    (1 - 1.98 x + 0.9801)^{-1/2}, omega = N/4 = 16384, N = 65536,
    M = 262144.  The stated Q = 64 does not resolve cos(16384 x); pass a
    resolving Q (about omega/2 plus a margin) for accuracy runs."""
    N = 65536
    f = Sum(Cosine(N / 4), GeneratingFunction(0.99))
    return SingleWorkload("cos16384_plus_genfn0.99", f, N, 262144, Q,
                          {"omega": N / 4, "t": 0.99})


def subset_indices(N: int = 65536, k: int = 512, seed: int = 2) -> np.ndarray:
    """Seeded random subset of coefficient indices for sampled parity."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, k, replace=False))


@dataclass
class SeriesBatch:
    """Batch of random finite Legendre series (true coefficients known)."""
    N: np.ndarray          # coefficients requested per function
    M: np.ndarray          # y-grid size per function
    Q: np.ndarray          # Abel nodes per function
    coeffs: list           # true coefficients per function (len N_b)


def batch_uneven(B: int = 4096, seed: int = 3, Q: int = 48,
                 n_lo: int = 256, n_hi: int = 8192) -> SeriesBatch:
    """Ragged batch: N_b = floor(exp(U(ln n_lo, ln n_hi))),
    c_{b,n} = Normal(0,1) / (n+1)^2 for n < N_b, M_b = 4 N_b, Q_b = Q."""
    rng = np.random.default_rng(seed)
    Nb = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), B))).astype(np.int64)
    Nb = np.clip(Nb, n_lo, n_hi)
    coeffs = []
    for b in range(B):
        n = np.arange(Nb[b], dtype=np.float64)
        coeffs.append(rng.standard_normal(Nb[b]) / (n + 1.0) ** 2)
    return SeriesBatch(Nb, 4 * Nb, np.full(B, Q, dtype=np.int32), coeffs)


def chebyshev_gauss_nodes(P: int) -> np.ndarray:
    """x_p = cos((2p+1) pi / (2P)), p = 0..P-1 (fixed sample grid of the
    Abel-as-GEMM workload)."""
    p = np.arange(P, dtype=np.float64)
    return np.cos((2 * p + 1) * np.pi / (2 * P))


def gemm_batch_coeffs(B: int, degree: int = 3000, seed: int = 4,
                      flat: bool = False) -> np.ndarray:
    """Band-limited random Legendre series for the fixed-grid workload:
    c_{b,n} = Normal(0,1) (n+1)^{-2} for n <= degree (flat=True: Normal(0,1)),
    returned as a [B][degree+1] float64 array."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((B, degree + 1))
    if not flat:
        c = c / (np.arange(degree + 1, dtype=np.float64) + 1.0) ** 2
    return c


@dataclass
class MixedStream:
    """Pareto-distributed batch of generating functions and exponentials."""
    N: np.ndarray
    kind: np.ndarray       # 0: generating function, 1: exponential
    param: np.ndarray      # t or a
    fp64: np.ndarray       # True: FP64 request, False: mixed-precision request


def mixed_stream(B: int = 65536, seed: int = 5, alpha: float = 1.2,
                 n_lo: int = 32, n_hi: int = 65536) -> MixedStream:
    """N_b from a Pareto(alpha) truncated to [n_lo, n_hi] by inversion,
    N_b = floor(n_lo (1 - u (1 - (n_lo/n_hi)^alpha))^{-1/alpha});
    even b: generating function with t ~ U(0.1, 0.999);
    odd b: e^{a x} with a ~ U(-20, 20); precision alternates FP64 / mixed."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, B)
    Nb = np.floor(n_lo * (1.0 - u * (1.0 - (n_lo / n_hi) ** alpha)) ** (-1.0 / alpha))
    Nb = np.clip(Nb, n_lo, n_hi).astype(np.int64)
    t = rng.uniform(0.1, 0.999, B)
    a = rng.uniform(-20.0, 20.0, B)
    kind = (np.arange(B) % 2).astype(np.int32)
    param = np.where(kind == 0, t, a)
    fp64 = (np.arange(B) // 2) % 2 == 0
    return MixedStream(Nb, kind, param, fp64)


def stream_grid(ms: MixedStream, b: int) -> int:
    """M_b of request b: 4 N_b, enlarged for a generating function so that
    the aliased tail t^{n+M} falls below 1e-13 (M_b >= N_b + ln(1e-13)/ln t
    + 1); even."""
    N = int(ms.N[b])
    M = 4 * N
    if ms.kind[b] == 0:
        t = float(ms.param[b])
        M = max(M, N + int(np.ceil(np.log(1e-13) / np.log(t))) + 1)
    return M + M % 2


def stream_rule(ms: MixedStream, b: int) -> dict:
    """The caller's choice of Abel rule for request b (an lc_abel_rule with
    no band and no breakpoints).  Generating function: 16-node panels
    graded toward x = 1 with ratio 0.2 and K = max(0, ceil(ln(d/4)/ln 0.2))
    levels, where d = (1-t)^2/(2t) is the distance of its singularity
    beyond x = 1 (about d/4 beyond t = 1 in the rule's variable at y = pi),
    so that the last panel is no wider than that distance.  e^{ax}: one
    panel of q = 16 nodes for |a| <= 8, 24 above."""
    if ms.kind[b] == 0:
        t = float(ms.param[b])
        d = (1.0 - t) ** 2 / (2.0 * t)
        K = max(0, int(np.ceil(np.log(d / 4.0) / np.log(0.2))))
        return {"q": 16, "grade_ratio": 0.2 if K else 0.0, "grade_levels": K}
    return {"q": 16 if abs(float(ms.param[b])) <= 8.0 else 24, "grade_ratio": 0.0, "grade_levels": 0}


def stream_function(ms: MixedStream, b: int):
    if ms.kind[b] == 0:
        return GeneratingFunction(float(ms.param[b]))
    return Exponential(float(ms.param[b]))
