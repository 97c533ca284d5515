"""Pins of the oracle's consistently integrated operator (section 3.3: 2r+1
Gauss points per direction instead of the r+1 of the fast evaluation).

* with r+1 points it is the standard operator (pinned elsewhere) exactly;
* Gauss exactness: on affine cells with coefficients of degree <= k every
  integrand is a polynomial of degree <= 3k per direction, integrated
  exactly by 2k+1 points, so 2k+1 and 3k+2 points agree to rounding while
  k+1 points do not (aliasing);
* its unit-vector matrix is symmetric positive definite.
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si


def _poly_problem(mesh, k):
    p = oracle.Problem(mesh, k)
    x, y, z = p.dof_coords()
    # nodal interpolants of polynomials of degree <= k are the polynomials
    p.set_coefficients(1.0 + 0.5 * x + 0.3 * y * z, 0.2 + 0.1 * x * x + 0.05 * y)
    return p


@pytest.mark.parametrize("k", [1, 2, 3])
def test_k_plus_one_points_is_the_standard_operator(k):
    p = oracle.Problem(si.terrain_mesh(3, 2, 2, g=2), k)
    p.set_coefficient_functions(*si.random_smooth_coefficients(1))
    x = si.random_vector(p.n_dofs, 2)
    np.testing.assert_array_equal(p.apply_q(x, k + 1), p.apply(x))


@pytest.mark.parametrize("k", [2, 3])
def test_gauss_exactness_on_affine_cells(k):
    m = si.box_mesh(2, 2, 2, periodic=(True, False, True), mapping=si.random_affine_mapping(4))
    p = _poly_problem(m, k)
    x = si.random_vector(p.n_dofs, 3)
    y_c = p.apply_q(x, 2 * k + 1)
    y_hi = p.apply_q(x, 3 * k + 2)
    y_fast = p.apply(x)
    scale = np.abs(y_hi).max()
    assert np.abs(y_c - y_hi).max() <= 1e-13 * scale
    assert np.abs(y_fast - y_hi).max() >= 1e-6 * scale      # the fast rule aliases


def test_matrix_symmetric_positive():
    m = si.box_mesh(2, 1, 2, periodic=(True, True, False), g=2,
                    mapping=si.random_affine_mapping(6))
    p = oracle.Problem(m, 1)
    p.set_coefficient_functions(*si.random_smooth_coefficients(5))
    n = p.n_dofs
    A = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = p.apply_q(e, 3)
        e[j] = 0.0
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
