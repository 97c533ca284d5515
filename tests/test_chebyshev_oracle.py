"""Pins of the oracle's Chebyshev preconditioner and Lanczos estimates
(section 3.1: a Chebyshev polynomial damping the eigenvalue range estimated
by the Lanczos process, for the symmetric positive-definite systems).

* residual polynomial: for a diagonal matrix with M = I, r - A z equals
  T_m((theta - A)/delta) / T_m(theta/delta) r, with numpy's Chebyshev T_m
  (a closed form of the recurrence);
* Lanczos: the Ritz values from CG coefficients lie inside the spectrum of
  M^-1 A and the extreme ones approach its extreme eigenvalues (dense
  generalized eigenvalues of (A, M) on a tiny mesh, M the block Jacobi).
"""
import numpy as np
import pytest
import scipy.linalg

import oracle
import synth_inputs as si
from oracle.solvers import chebyshev_apply, lanczos_bounds


@pytest.mark.parametrize("degree", [1, 2, 5, 9])
def test_residual_is_scaled_chebyshev_polynomial(degree):
    lam = np.linspace(0.3, 4.0, 40)
    r = si.random_vector(40, 3)
    lo, hi = 0.25, 4.2
    z = chebyshev_apply(lambda v: lam * v, lambda v: v.copy(), r, lo, hi, degree)
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    T = np.polynomial.chebyshev.Chebyshev.basis(degree)
    expect = T((theta - lam) / delta) / T(theta / delta) * r
    np.testing.assert_allclose(r - lam * z, expect, rtol=0, atol=1e-13 * np.abs(r).max())


def test_lanczos_bounds_inside_and_converging():
    m = si.terrain_mesh(2, 1, 2, g=2)
    p = oracle.Problem(m, 1)
    p.set_coefficient_functions(*si.terrain_coefficients())
    A = p.assemble_dense()
    n, nd = p.n_dofs, p.nd
    M = np.zeros((n, n))
    for c in range(p.n_cells):
        M[c * nd:(c + 1) * nd, c * nd:(c + 1) * nd] = p.bj_sep_block(c)
    ev = scipy.linalg.eigh(A, M, eigvals_only=True)
    b = si.random_vector(n, 9)
    lo, hi = lanczos_bounds(p.apply, p.bj_apply, b, 12)
    assert ev[0] * (1 - 1e-10) <= lo and hi <= ev[-1] * (1 + 1e-10)
    lo2, hi2 = lanczos_bounds(p.apply, p.bj_apply, b, n - 1)
    assert abs(hi2 - ev[-1]) <= 1e-6 * ev[-1] and abs(lo2 - ev[0]) <= 1e-6 * ev[-1]
