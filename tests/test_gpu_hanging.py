"""GPU parity on non-conforming meshes (2:1 hanging faces, the paper's second
mesh, section 3) against the oracle, whose quarter-face terms are pinned in
test_hanging_oracle.py: the operator (FP64 to 1e-12 normwise and max-abs,
FP32 to 2e-6, residual form, face part, with and without the affine
compression), its dense matrix by unit vectors, the separable block Jacobi
with the quarter penalties at non-conforming ends, the volume diagonals,
solves against the oracle's 1e-13 solution, the error paths of the set-up,
and the features the mesh does not support."""
import numpy as np
import pytest

import oracle
import synth_inputs as si
from helpers import gpu_context, normwise, problem, to_dev

pytestmark = pytest.mark.gpu


def _hx():
    import paper_2505_00384_amd as hx
    return hx


def _check(y, ref, tol=1e-12):
    e2, einf = normwise(y, ref)
    assert e2 <= tol and einf <= tol, (e2, einf)


MESHES = [
    ("2x2x2-periodic", lambda: si.refined_mesh(2, 2, 2, ((0, 1), (0, 1), (0, 1)))),
    ("3x3x2-neumann", lambda: si.refined_mesh(3, 3, 2, ((1, 2), (0, 2), (0, 1)), periodic=(False,) * 3)),
    ("2x1x2-sheared", lambda: si.refined_mesh(2, 1, 2, ((0, 1), (0, 1), (1, 2)),
                                              periodic=(True, True, False),
                                              mapping=si.random_affine_mapping(3))),
    ("terrain-4x2x2-g3", lambda: si.refined_terrain_mesh(4, 2, 2, g=3, region=((1, 3), (0, 1), (0, 1)))),
    ("wavy-2-g2", lambda: si.refined_mesh(2, 2, 2, ((0, 1), (0, 2), (0, 1)), g=2,
                                          mapping=si.wavy_mapping(0.04))),
]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_hanging_operator_parity(k):
    hx = _hx()
    for name, mk in MESHES:
        m = mk()
        if k == 4 and m.n_cells > 16:
            continue
        print(f"[hanging] k={k} mesh={name} cells={m.n_cells} quarters={m.hang.shape[0]}", flush=True)
        p = problem(m, k, coef="terrain" if name.startswith("terrain") else "random", seed=k)
        ctx = gpu_context(p)
        x = si.random_vector(p.n_dofs, 40 + k)
        xd = to_dev(x)
        ref = p.apply(x)
        _check(ctx.apply_operator(xd).cpu().numpy(), ref)
        # the general data layout gives the same
        ctx.set_cell_compression(False)
        _check(ctx.apply_operator(xd).cpu().numpy(), ref)
        ctx.set_cell_compression(True)
        # face part, residual form, FP32
        _check(ctx.apply_operator_part(hx.HX_PART_FACE, xd).cpu().numpy(), p.apply(x, oracle.OR_FACE))
        b = si.random_vector(p.n_dofs, 70 + k)
        r = ctx.residual(to_dev(b), xd).cpu().numpy()
        assert np.abs(r - (b - ref)).max() <= 1e-12 * np.abs(b - ref).max()
        y32 = ctx.apply_operator(xd.float()).cpu().numpy()
        assert np.linalg.norm(y32 - ref) <= 2e-6 * np.linalg.norm(ref)
        # bitwise repeatable
        y1 = ctx.apply_operator(xd).cpu().numpy()
        y2 = ctx.apply_operator(xd).cpu().numpy()
        assert np.array_equal(y1, y2)
        ctx.close()


def test_hanging_dense_matrix_by_unit_vectors():
    import torch
    m = MESHES[0][1]()
    p = problem(m, 2, seed=3)
    ctx = gpu_context(p)
    n = p.n_dofs
    E = torch.eye(n, dtype=torch.float64, device="cuda:0")
    A = np.stack([ctx.apply_operator(E[j].contiguous()).cpu().numpy() for j in range(n)], axis=1)
    ref = p.assemble_dense()
    assert np.abs(A - ref).max() <= 1e-12 * np.abs(ref).max()
    ctx.close()


@pytest.mark.parametrize("k", [1, 2, 4])
def test_hanging_block_jacobi_and_diagonals(k):
    hx = _hx()
    for name, mk in MESHES[1:4]:
        p = problem(mk(), k, coef="terrain" if name.startswith("terrain") else "random", seed=k)
        ctx = gpu_context(p)
        r = si.random_vector(p.n_dofs, 9)
        z = ctx.apply_preconditioner(to_dev(r)).cpu().numpy()
        zr = p.bj_apply(r)
        assert np.linalg.norm(z - zr) <= 1e-11 * np.linalg.norm(zr), name
        inv = ctx.debug_export(hx.HX_EXPORT_INV_DIAG, (2, p.n_dofs))
        for row, stiff in ((0, True), (1, False)):
            ref = p.cell_diagonal(stiff=stiff)
            assert np.abs(1.0 / inv[row] - ref).max() <= 1e-12 * np.abs(ref).max(), (name, stiff)
        ctx.close()


def test_hanging_solves_against_oracle():
    """CG with block Jacobi and the paper's Helmholtz diagonal, FGMRES and the
    mixed form on a refined terrain channel (Q3) against the oracle's 1e-13
    solution; the oracle's residual of each GPU solution is 1e-8."""
    hx = _hx()
    m = si.refined_terrain_mesh(8, 2, 4, g=3)
    p = problem(m, 3, coef="terrain")
    b = si.rhs_terrain(4)(*p.dof_coords())
    xs, info = oracle.solvers.cg(p.apply, b, precond=p.bj_apply, rtol=1e-13, max_iter=5000)
    assert info.converged
    ctx = gpu_context(p)
    bd = to_dev(b)
    nb = np.linalg.norm(b)
    for name, prm in [("cg_bj", hx.default_params(method=0, rtol=1e-8)),
                      ("cg_helmholtz", hx.default_params(method=0, rtol=1e-8, max_iter=20000,
                                                         pc=hx.HX_PC_HELMHOLTZ_DIAG)),
                      ("fgmres_bj", hx.default_params(method=1, restart=30, rtol=1e-8)),
                      ("mixed", hx.default_params(method=1, restart=10, rtol=1e-8, mixed=1, inner_iters=16))]:
        x, inf = ctx.solve(bd, params=prm)
        x = x.cpu().numpy()
        err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
        res = np.linalg.norm(b - p.apply(x)) / nb
        print(f"[hanging solve] {name}: {inf['iters']} it, residual {inf['true_rel_res']:.2e}, "
              f"oracle residual {res:.2e}, error {err:.2e}", flush=True)
        assert inf["status"] == hx.HX_OK and inf["true_rel_res"] <= 1e-8
        assert res <= 1.001e-8 and err <= 1e-6, (name, res, err)
    ctx.close()


def test_hanging_setup_errors_and_unsupported_features():
    import torch
    hx = _hx()
    m = MESHES[1][1]()
    p = problem(m, 1)
    ctx = hx.HelmDG(0)
    # marked faces without records
    with pytest.raises(hx.HXError) as e:
        ctx.setup_mesh(1, m.nodes, m.nbr, 1)
    assert e.value.status == hx.HX_ERR_MESH
    # a record missing (the coarse face loses a quarter)
    with pytest.raises(hx.HXError) as e:
        ctx.setup_mesh(1, m.nodes, m.nbr, 1, hang=m.hang[1:])
    assert e.value.status == hx.HX_ERR_MESH
    # a quarter listed twice
    bad = m.hang.copy()
    q = np.nonzero(bad[:, 0] == bad[0, 0])[0]
    bad[q[1], 3] = bad[q[0], 3]
    with pytest.raises(hx.HXError) as e:
        ctx.setup_mesh(1, m.nodes, m.nbr, 1, hang=bad)
    assert e.value.status == hx.HX_ERR_MESH
    ctx.setup_mesh(1, m.nodes, m.nbr, 1, hang=m.hang)
    ctx.set_coefficients(p.alpha, p.beta, 2.0)
    ones = torch.ones(ctx.n_dofs, dtype=torch.float64, device="cuda:0")
    with pytest.raises(hx.HXError) as e:
        ctx.set_pressure_system(ones, ones, 1.4, 1.0)
    assert e.value.status == hx.HX_ERR_STATE
    with pytest.raises(hx.HXError) as e:
        ctx.set_consistent(ones, ones)
    assert e.value.status == hx.HX_ERR_STATE
    c2 = hx.HelmDG(0)
    c2.setup_mesh(1, m.nodes, m.nbr, 1, hang=m.hang)
    c2.set_coefficients(p.alpha, p.beta, 2.0)
    with pytest.raises(hx.HXError) as e:
        ctx.set_multigrid(c2, np.zeros(m.n_cells, np.int32), np.zeros(m.n_cells, np.int32))
    assert e.value.status == hx.HX_ERR_STATE
    c2.close()
    # the penalty factor can change after set-up (quarter penalties follow)
    ctx.set_coefficients(p.alpha, p.beta, 3.0)
    p3 = oracle.Problem(m, 1, alpha=p.alpha, beta=p.beta, P=3.0)
    x = si.random_vector(p.n_dofs, 2)
    _check(ctx.apply_operator(to_dev(x)).cpu().numpy(), p3.apply(x))
    assert np.linalg.norm(ctx.apply_preconditioner(to_dev(x)).cpu().numpy() - p3.bj_apply(x)) <= \
        1e-11 * np.linalg.norm(p3.bj_apply(x))
    ctx.close()
