"""Pins of the oracle's geometric multigrid (section 3.1: CG preconditioned by
geometric multigrid for the SPD systems, Chebyshev smoothing).  Each pin
comes from the mathematics of nested spaces, not from the oracle itself:

* prolongation reproduces every polynomial of total degree <= k on nested
  affine meshes (the coarse space is a subspace of the fine one);
* restriction is the transpose of prolongation, pinned by the Galerkin
  identity R M_fine P = M_coarse, exact for the mass matrix on nested affine
  meshes (both levels integrate degree 2k exactly);
* for continuous fields the same identity holds for the whole interior-penalty
  operator with constant coefficients and wall boundaries: fine faces inside a
  coarse cell see no jump of either function, the coarse faces split into
  fine ones with the same integrands, and penalties multiply zero jumps;
* the V-cycle with the same polynomial before and after the coarse correction
  is symmetric and positive definite;
* CG with one V-cycle per iteration needs far fewer iterations than CG with
  block Jacobi on the terrain channel.
"""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from oracle import multigrid as mg
from oracle import solvers
from helpers import terrain_hierarchy, oracle_levels


def _nested(nx, ny, nz, k, seed, periodic=(False, False, False)):
    f = si.random_affine_mapping(seed)
    fine = oracle.Problem(si.box_mesh(2 * nx, 2 * ny, 2 * nz, periodic=periodic, mapping=f), k)
    coarse = oracle.Problem(si.box_mesh(nx, ny, nz, periodic=periodic, mapping=f), k)
    return fine, coarse, si.refinement_parents(nx, ny, nz)


def _poly(k, seed):
    rng = np.random.default_rng(seed)
    terms = [(a, b, c, rng.standard_normal()) for a in range(k + 1) for b in range(k + 1 - a)
             for c in range(k + 1 - a - b)]
    return lambda x, y, z: sum(w * x ** a * y ** b * z ** c for a, b, c, w in terms)


def test_octant_embeddings_partition_of_unity_and_nodes():
    for k in range(1, 9):
        E = mg.octant_embeddings(k)
        assert np.abs(E.sum(axis=2) - 1.0).max() < 1e-13
        # the lower half's first node and the upper half's last node are parent nodes
        assert np.abs(E[0, 0] - np.eye(k + 1)[0]).max() < 1e-14
        assert np.abs(E[1, -1] - np.eye(k + 1)[-1]).max() < 1e-14


@pytest.mark.parametrize("k", [1, 2, 4, 6])
@pytest.mark.parametrize("dims", [(3, 2, 1), (1, 2, 2)])
def test_prolongation_reproduces_polynomials(k, dims):
    fine, coarse, (parent, octant) = _nested(*dims, k, seed=k)
    f = _poly(k, seed=7 * k + dims[0])
    xc = f(*coarse.dof_coords())
    xf = mg.prolong(k, parent, octant, xc)
    ref = f(*fine.dof_coords())
    assert np.abs(xf - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("k", [1, 3, 4])
def test_restricted_fine_mass_is_coarse_mass(k):
    fine, coarse, (parent, octant) = _nested(2, 1, 2, k, seed=3, periodic=(True, False, True))
    for p in (fine, coarse):
        p.set_coefficients(np.full(p.n_dofs, 1.3), np.zeros(p.n_dofs))
    xc = si.random_vector(coarse.n_dofs, 5)
    lhs = mg.restrict(k, parent, octant, fine.apply(mg.prolong(k, parent, octant, xc)),
                      coarse.n_cells)
    rhs = coarse.apply(xc)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


@pytest.mark.parametrize("k", [1, 2, 4])
def test_restricted_fine_operator_on_continuous_fields(k):
    fine, coarse, (parent, octant) = _nested(2, 2, 1, k, seed=11)
    for p in (fine, coarse):
        p.set_coefficients(np.full(p.n_dofs, 0.7), np.full(p.n_dofs, 0.3))
    u = _poly(k, seed=3 + k)(*coarse.dof_coords())
    lhs = mg.restrict(k, parent, octant, fine.apply(mg.prolong(k, parent, octant, u)),
                      coarse.n_cells)
    rhs = coarse.apply(u)
    assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(rhs).max()
    # a discontinuous field sees the finer penalty: the identity must fail
    v = si.random_vector(coarse.n_dofs, 2)
    lv = mg.restrict(k, parent, octant, fine.apply(mg.prolong(k, parent, octant, v)),
                     coarse.n_cells)
    assert np.abs(lv - coarse.apply(v)).max() > 1e-3 * np.abs(lv).max()


def test_vcycle_symmetric_positive_definite():
    probs, maps = terrain_hierarchy(8, 4, 4, 3, 2)
    levels = oracle_levels(probs, maps)
    n = probs[0].n_dofs
    a, b = si.random_vector(n, 1), si.random_vector(n, 2)
    Va, Vb = mg.vcycle(levels, a), mg.vcycle(levels, b)
    assert abs(Va @ b - a @ Vb) <= 1e-12 * np.linalg.norm(Va) * np.linalg.norm(b)
    for v, Vv in ((a, Va), (b, Vb)):
        assert v @ Vv > 0


def test_mg_cg_beats_block_jacobi():
    probs, maps = terrain_hierarchy(16, 4, 8, 3, 2)
    levels = oracle_levels(probs, maps)
    p = probs[0]
    b = p.load_vector(si.rhs_terrain(0))
    x_mg, info_mg = mg.mg_cg(levels, b, rtol=1e-8)
    x_bj, info_bj = solvers.cg(p.apply, b, precond=p.bj_apply, rtol=1e-8)
    assert info_mg.converged and info_mg.true_rel_res <= 1.1e-8
    assert info_mg.iters <= 10 and info_mg.iters * 3 <= info_bj.iters, (info_mg.iters, info_bj.iters)
    assert np.linalg.norm(x_mg - x_bj) <= 1e-6 * np.linalg.norm(x_bj)


def test_pins_catch_planted_mistakes(monkeypatch):
    """Plausible mistakes planted in the oracle (on the CPU) fail the pins
    above: the two halves of the embedding swapped, the x and z octant bits
    exchanged, and a cycle without post-smoothing (not symmetric)."""
    k = 2
    fine, coarse, (parent, octant) = _nested(3, 2, 1, k, seed=2)
    f = _poly(k, seed=5)
    xc = f(*coarse.dof_coords())
    ref = f(*fine.dof_coords())
    scale = np.abs(ref).max()
    assert np.abs(mg.prolong(k, parent, octant, xc) - ref).max() <= 1e-12 * scale
    good = mg.octant_embeddings
    monkeypatch.setattr(mg, "octant_embeddings", lambda kk: good(kk)[::-1].copy())
    assert np.abs(mg.prolong(k, parent, octant, xc) - ref).max() > 1e-3 * scale
    monkeypatch.setattr(mg, "octant_embeddings", good)
    swapped = ((octant & 1) << 2) | (octant & 2) | ((octant >> 2) & 1)
    assert np.abs(mg.prolong(k, parent, swapped, xc) - ref).max() > 1e-3 * scale
    # a V-cycle that skips the post-smoothing is not symmetric
    probs, maps = terrain_hierarchy(8, 4, 4, 2, 2)
    levels = oracle_levels(probs, maps)

    def pre_only(b):
        L, C = levels
        x = L.smooth(b)
        r = b - L.prob.apply(x)
        bc = mg.restrict(k, L.parent, L.octant, r, C.prob.n_cells)
        return x + mg.prolong(k, L.parent, L.octant, C.smooth(bc))
    n = probs[0].n_dofs
    a, b = si.random_vector(n, 1), si.random_vector(n, 2)
    Va, Vb = mg.vcycle(levels, a), mg.vcycle(levels, b)
    assert abs(Va @ b - a @ Vb) <= 1e-12 * np.linalg.norm(Va) * np.linalg.norm(b)
    Pa, Pb = pre_only(a), pre_only(b)
    assert abs(Pa @ b - a @ Pb) > 1e-6 * np.linalg.norm(Pa) * np.linalg.norm(b)
