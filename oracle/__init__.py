"""CPU oracle for the Legendre-coefficient method (arXiv 1106.0463).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
the CPU-baseline leg of the benchmark may import this package.  It shares no
code with the HIP library and imports nothing from it.

* :mod:`oracle.definition` -- eq. (2.3) by brute-force Gauss-Legendre
  quadrature with the three-term recurrence (long double, O(N K)).
* :mod:`oracle.method` -- the paper's discretized method step by step
  (Abel-type transform eqs. (2.5)/(2.14), trapezoid rule for eq. (2.4),
  c_n = (2n+1) a_n), long double, with a plain O(M N) Fourier sum; also the
  composite Abel rule (breakpoints, grading toward x = 1, per-row node
  counts).

The closed-form coefficients and Abel transforms that pin the two modules
above live with the tests (``tests/closed_forms.py``), not in this package.

Pins (the tests under ``tests/test_oracle_*.py``): textbook Gauss-Legendre
nodes, monomial exactness, f = P_m, the generating function eq. (2.2),
e^{ax} through modified spherical Bessel functions, |x|^{3/2} against the
True column of Table 1, reconstruction by eq. (2.1), mpmath brute-force
quadrature of eq. (2.3) and eq. (2.14), polynomial exactness of the
discretized method and its aliasing law, and the subset transform
(eq. (2.4) at listed indices) and the [M/2][Q] sample builder against
closed forms and an independent Gauss-Legendre routine.
"""
from ._lib import build, load, threads  # noqa: F401
from .definition import (gauss_legendre, legendre_coeffs,  # noqa: F401
                         legendre_coeffs_from_samples,
                         legendre_coeffs_piecewise, legendre_eval)
from .method import (abel_fhat, abel_node_set, abel_nodes, abel_phi, abel_phi_rule,  # noqa: F401
                     abel_rule_cuts, abel_rule_ladder, abel_rule_node_count, abel_rule_panel_q,
                     abel_rule_row_q,
                     coeffs_from_fhat, fhat_from_phi, fourier_coeffs, fourier_coeffs_at,
                     method_coeffs, method_coeffs_2d, method_coeffs_at, method_coeffs_from_samples,
                     method_coeffs_rule,
                     positive_half_samples, y_grid)
