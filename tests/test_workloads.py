"""The seeded input generators: function families against independent
evaluations, and reproducibility of the seeded recipes."""
import numpy as np
from numpy.polynomial import legendre as npleg

import workloads as W


def test_legendre_series_clenshaw_matches_numpy_legval():
    c = np.random.default_rng(0).standard_normal(300) / (np.arange(300) + 1.0)
    x = np.linspace(-1, 1, 257)
    got = W.LegendreSeries(c)(x)
    ref = npleg.legval(x, c)
    assert np.max(np.abs(got - ref)) < 1e-13
    got_ld = W.LegendreSeries(c)(x.astype(np.longdouble))
    assert got_ld.dtype == np.longdouble
    assert np.max(np.abs(got_ld.astype(float) - ref)) < 1e-13


def test_generating_function_form():
    x = np.linspace(-1, 1, 101)
    for t in (0.1, 0.5, 0.99):
        assert np.allclose(W.GeneratingFunction(t)(x), (1 - 2 * x * t + t * t) ** -0.5,
                           rtol=1e-12, atol=0)


def test_seeded_recipes_are_reproducible():
    a = W.batch_uneven(B=64)
    b = W.batch_uneven(B=64)
    assert np.array_equal(a.N, b.N)
    assert all(np.array_equal(x, y) for x, y in zip(a.coeffs, b.coeffs))
    assert a.N.min() >= 256 and a.N.max() <= 8192
    assert np.array_equal(a.M, 4 * a.N)
    ms = W.mixed_stream(B=1000)
    assert ms.N.min() >= 32 and ms.N.max() <= 65536
    assert np.all((ms.param[ms.kind == 0] > 0.1) & (ms.param[ms.kind == 0] < 0.999))
    s = W.subset_indices()
    assert s.size == 512 and np.unique(s).size == 512 and s.max() < 65536


def test_chebyshev_gauss_nodes():
    x = W.chebyshev_gauss_nodes(8)
    assert np.allclose(np.polynomial.chebyshev.chebval(x, [0] * 8 + [1]), 0, atol=1e-14)
