"""Pins of the oracle's volume diagonals, the matrices whose inverses are the
paper's diagonal preconditioners (section 3.1: the "Helmholtz
preconditioner" inverts the diagonal of the volume terms of S~, mass plus
dt-scaled stiffness; the "internal-energy" variant keeps the mass alone).

* Cartesian closed form: on the affine periodic cube with constant
  coefficients the volume diagonal is the diagonal of
  alpha h^3 M(x)M(x)M + beta h (K(x)M(x)M + M(x)K(x)M + M(x)M(x)K), with the 1-D
  reference mass M and volume stiffness K built here from numpy's Gauss rule
  and monomial-fitted Lagrange polynomials.
* Another route through the oracle: on curved cells with variable
  coefficients it equals the diagonal of the matrix of the cell-only operator
  applied to unit vectors (the paper's own way of building a matrix from an
  operator action), and with beta = 0 the same holds for the mass diagonal.
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from test_oracle_pins import _np_lagrange, _np_rules


def _ref_1d(k):
    n = k + 1
    xq, wq, xl = _np_rules(n)
    M = np.zeros((n, n)); K = np.zeros((n, n))
    for x, w in zip(xq, wq):
        v, d = _np_lagrange(xl, x)
        M += w * np.outer(v, v); K += w * np.outer(d, d)
    return np.diag(M), np.diag(K)


@pytest.mark.parametrize("k,nc", [(2, 3), (4, 2), (1, 2)])
def test_cartesian_closed_form(k, nc):
    alpha, beta, h = 1.7, 0.3, 1.0 / nc
    p = oracle.Problem(si.cube_mesh(nc), k)
    p.set_coefficient_functions(*si.const_coefficients(alpha, beta))
    m, kk = _ref_1d(k)
    n = k + 1
    ref_m = np.zeros(n ** 3); ref_a = np.zeros(n ** 3)
    for l in range(n):
        for j in range(n):
            for i in range(n):
                mm = m[i] * m[j] * m[l]
                ref_m[i + n * (j + n * l)] = alpha * h ** 3 * mm
                ref_a[i + n * (j + n * l)] = alpha * h ** 3 * mm + beta * h * (
                    kk[i] * m[j] * m[l] + m[i] * kk[j] * m[l] + m[i] * m[j] * kk[l])
    dm = p.cell_diagonal(stiff=False).reshape(p.n_cells, -1)
    da = p.cell_diagonal(stiff=True).reshape(p.n_cells, -1)
    for c in range(p.n_cells):
        np.testing.assert_allclose(dm[c], ref_m, rtol=1e-13)
        np.testing.assert_allclose(da[c], ref_a, rtol=1e-13)


@pytest.mark.parametrize("mesh,k", [("terrain", 2), ("wavy", 3)])
def test_equals_unit_vector_matrix_of_cell_operator(mesh, k):
    if mesh == "terrain":
        msh = si.terrain_mesh(2, 1, 2, g=2)
        fa, fb = si.terrain_coefficients()
    else:
        msh = si.wavy_cube_mesh(2, g=2)
        fa, fb = si.random_smooth_coefficients(3)
    p = oracle.Problem(msh, k)
    p.set_coefficient_functions(fa, fb)
    A = p.matrix_by_unit_vectors(oracle.OR_CELL)
    d = p.cell_diagonal(stiff=True)
    np.testing.assert_allclose(d, np.diag(A), rtol=1e-12, atol=1e-14 * np.abs(d).max())
    assert (d > 0).all()
    # mass alone: the same operator with beta = 0
    x, y, z = p.dof_coords()
    p.set_coefficients(fa(x, y, z), np.zeros(p.n_dofs))
    A0 = p.matrix_by_unit_vectors(oracle.OR_CELL)
    p.set_coefficients(fa(x, y, z), fb(x, y, z))
    dm = p.cell_diagonal(stiff=False)
    np.testing.assert_allclose(dm, np.diag(A0), rtol=1e-12, atol=1e-14 * np.abs(dm).max())
    assert (dm > 0).all() and (d > dm).all()


# ---------------------------------------------------------------------------
# cell mass blocks: the block-diagonal matrix section 3.3 inverts by its
# tensor-product factors
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k,nc", [(2, 2), (4, 1), (3, 2)])
def test_mass_block_cartesian_closed_form(k, nc):
    alpha, h = 1.3, 1.0 / nc
    p = oracle.Problem(si.cube_mesh(nc), k)
    p.set_coefficient_functions(*si.const_coefficients(alpha, 0.2))
    n = k + 1
    xq, wq, xl = _np_rules(n)
    M1 = np.zeros((n, n))
    for x, w in zip(xq, wq):
        v, _ = _np_lagrange(xl, x)
        M1 += w * np.outer(v, v)
    ref = alpha * h ** 3 * np.kron(M1, np.kron(M1, M1))   # z slowest, x fastest
    for c in range(p.n_cells):
        np.testing.assert_allclose(p.mass_block(c), ref, rtol=1e-13, atol=1e-15 * np.abs(ref).max())
    r = si.random_vector(p.n_dofs, 1)
    z = p.mass_block_apply(r)
    for c in range(p.n_cells):
        s = slice(c * n ** 3, (c + 1) * n ** 3)
        np.testing.assert_allclose(ref @ z[s], r[s], rtol=1e-10, atol=1e-12 * np.abs(r).max())


def test_mass_block_is_the_cell_operator_block_without_stiffness():
    msh = si.terrain_mesh(2, 1, 2, g=2)
    fa, fb = si.terrain_coefficients()
    p = oracle.Problem(msh, 2)
    x, y, z = (lambda t: t)(p.dof_coords())
    p.set_coefficients(fa(x, y, z), np.zeros(p.n_dofs))
    A0 = p.matrix_by_unit_vectors(oracle.OR_CELL)
    nd = p.nd
    for c in range(p.n_cells):
        s = slice(c * nd, (c + 1) * nd)
        blk = A0[s, s]
        np.testing.assert_allclose(p.mass_block(c), blk, rtol=1e-12, atol=1e-14 * np.abs(blk).max())
        # nothing outside the cell's own block
        assert np.abs(np.delete(A0[s], np.arange(c * nd, (c + 1) * nd), axis=1)).max() == 0.0
