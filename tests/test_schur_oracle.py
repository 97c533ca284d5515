"""Pins of the oracle's velocity-pressure coupling (section 2: A U + B P = F,
C U + D P = G and the pressure system D P + C A^-1 (F - B P) = G), read with
central fluxes.  Each pin comes from the mathematics, not from the oracle:

* adjointness: on affine cells (exact quadrature) with a constant weight
  hr = c, summation by parts gives c(u, q) = -c b(q, u), i.e. C = -c B^T,
  for random u, q, with periodic and wall boundaries (the own trace in B and
  no flux in C on walls make the boundary terms cancel);
* B of a linear pressure a.x is tau a_c times the load vector of 1
  (the gradient of a smooth field tested against the basis);
* C of a constant velocity on a periodic affine mesh vanishes;
* with a constant hr the pressure system is symmetric positive definite
  (S = D + c B^T A^-1 B), with a variable hr it is not symmetric;
* consistency: on periodic cubes S applied to a smooth periodic p approaches
  the load vector of p/(gamma-1) - tau^2 hr/rho lap p as the mesh is refined;
* the fixed point (h re-evaluated from the previous iterate) converges to a
  state p* built to be its fixed point.
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from oracle.core import PressureSystem
from helpers import constructed_pressure_state, oracle_fixed_point

AFFINE = [
    ("cube3-periodic", lambda: si.cube_mesh(3)),
    ("box-walls-z", lambda: si.box_mesh(3, 2, 2, periodic=(True, True, False),
                                        mapping=si.random_affine_mapping(3))),
    ("box-walls-all", lambda: si.box_mesh(2, 2, 3, periodic=(False, False, False),
                                          mapping=si.random_affine_mapping(5))),
]


@pytest.mark.parametrize("name,mk", AFFINE, ids=[a[0] for a in AFFINE])
@pytest.mark.parametrize("k", [1, 2, 3])
def test_divergence_is_minus_weighted_gradient_transpose(name, mk, k):
    p = oracle.Problem(mk(), k)
    n = p.n_dofs
    u = si.random_vector(3 * n, 1).reshape(3, n)
    q = si.random_vector(n, 2)
    c, tau = 1.7, 0.3
    hr = np.full(n, c)
    lhs = p.div_apply(u, hr, tau) @ q
    rhs = -c * np.sum(p.grad_apply(q, tau) * u)
    scale = tau * c * np.linalg.norm(u) * np.linalg.norm(q)
    assert abs(lhs - rhs) <= 1e-13 * scale, (lhs, rhs)


LINEAR = [  # meshes on which a.x is continuous across every interior face
    ("box-walls-all", AFFINE[2][1], np.array([0.7, -1.3, 0.4])),
    ("box-walls-z", lambda: si.box_mesh(3, 2, 2, periodic=(True, True, False)),
     np.array([0.0, 0.0, 0.4])),
]


@pytest.mark.parametrize("name,mk,a", LINEAR, ids=[c[0] for c in LINEAR])
@pytest.mark.parametrize("k", [1, 3])
def test_gradient_of_linear_pressure(name, mk, a, k):
    p = oracle.Problem(mk(), k)
    x, y, z = p.dof_coords()
    pv = a[0] * x + a[1] * y + a[2] * z
    tau = 0.25
    g = p.grad_apply(pv, tau)
    ones = p.load_vector(lambda X, Y, Z: np.ones_like(X))
    for c in range(3):
        np.testing.assert_allclose(g[c], tau * a[c] * ones, rtol=0, atol=1e-13 * np.abs(ones).max())


@pytest.mark.parametrize("k", [1, 2])
def test_divergence_of_constant_velocity_periodic(k):
    p = oracle.Problem(si.box_mesh(3, 2, 2, mapping=si.random_affine_mapping(7)), k)
    n = p.n_dofs
    u = np.stack([np.full(n, 0.3), np.full(n, -1.1), np.full(n, 0.8)])
    q = p.div_apply(u, np.full(n, 2.5), 0.5)
    assert np.abs(q).max() <= 1e-13 * 2.5 * 0.5


def _dense(apply, n):
    S = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        S[:, j] = apply(e)
        e[j] = 0.0
    return S


def test_pressure_system_symmetric_with_constant_hr():
    m = si.box_mesh(2, 2, 2, periodic=(True, True, False), mapping=si.random_affine_mapping(2))
    p = oracle.Problem(m, 1)
    x, y, z = p.dof_coords()
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x) * np.cos(np.pi * z)
    h = 2.0 / rho                                  # h rho = 2 everywhere
    sysm = PressureSystem(m, 1, rho, h, gamma=1.4, tau=0.2)
    S = _dense(sysm.apply, p.n_dofs)
    assert np.abs(S - S.T).max() <= 1e-13 * np.abs(S).max()
    assert np.linalg.eigvalsh(0.5 * (S + S.T)).min() > 0
    # a variable h rho makes it non-symmetric
    sysv = PressureSystem(m, 1, rho, 1.0 + 0.5 * z, gamma=1.4, tau=0.2)
    Sv = _dense(sysv.apply, p.n_dofs)
    assert np.abs(Sv - Sv.T).max() >= 1e-3 * np.abs(Sv).max()


def test_pressure_system_consistency():
    """S p -> load vector of p/(gamma-1) + tau^2 (hr/rho) 8 pi^2 p for
    p = sin(2 pi x) sin(2 pi y) on periodic cubes (rho = 1, h = hr = 0.8)."""
    gamma, tau, h = 1.4, 0.05, 0.8
    lam = 1.0 / (gamma - 1.0) + tau ** 2 * h * 8 * np.pi ** 2
    f = lambda X, Y, Z: np.sin(2 * np.pi * X) * np.sin(2 * np.pi * Y)
    errs = []
    for nc in (4, 8):
        m = si.cube_mesh(nc)
        p = oracle.Problem(m, 2)
        x, y, z = p.dof_coords()
        n = p.n_dofs
        sysm = PressureSystem(m, 2, np.ones(n), np.full(n, h), gamma, tau)
        Sp = sysm.apply(f(x, y, z))
        ref = p.load_vector(lambda X, Y, Z: lam * f(X, Y, Z))
        errs.append(np.linalg.norm(Sp - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.05 and errs[1] < errs[0] / 3, errs


def test_fixed_point_converges_to_constructed_state():
    m = si.terrain_mesh(4, 2, 3, g=4)
    rho, F, G, p_bg, p_star, tau = constructed_pressure_state(m, 4, 1.4)
    errs = [np.linalg.norm(oracle_fixed_point(m, 4, rho, F, G, p_bg, 1.4, tau, it) - p_star)
            / np.linalg.norm(p_star) for it in (1, 5)]
    assert errs[0] < 1e-2 and errs[1] < 1e-9, errs


def test_cell_restricted_system_equals_full():
    """S p on sampled cells from their two-layer stencil (dense mass-block
    solves) equals the full composition: the form the full-size GPU test
    samples."""
    m = si.terrain_mesh(4, 2, 3, g=4)
    p = oracle.Problem(m, 4)
    x, y, z = p.dof_coords()
    fr, fh = si.terrain_pressure_fields()
    sysm = PressureSystem(m, 4, fr(x, y, z), fh(x, y, z), 1.4, 1.0)
    pv = si.random_vector(p.n_dofs, 3)
    full = sysm.apply(pv).reshape(m.n_cells, -1)
    cells = np.array([0, 5, 11, 23])
    part = sysm.apply_cells(pv, cells)
    assert np.abs(part - full[cells]).max() <= 1e-13 * np.abs(full).max()
