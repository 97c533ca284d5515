"""Exact inverse of the alpha-weighted cell mass blocks on the GPU (the
tensor-product inverse of section 3.3, M_K^{-1} = B3^{-1} diag(1/m_K) B3^{-T}):
compared with the oracle's dense Cholesky solve of every block (pinned in
test_diag_oracle.py), in FP64 and FP32, on curved and affine meshes of
degrees 1 to 7 and a ragged cell count; then used as a CG / FGMRES
preconditioner, where with beta = 0 the operator is the block mass matrix
itself and one CG step solves the system."""
import numpy as np
import pytest

import synth_inputs as si
from helpers import TINY, gpu_context, problem, to_dev

pytestmark = pytest.mark.gpu


def _hx():
    import paper_2505_00384_amd as hx
    return hx


CASES = [(name, mk, k) for (name, mk) in TINY for k in (1, 2)] + [
    ("terrain-4x2x3-g4", lambda: si.terrain_mesh(4, 2, 3, g=4), 4),
    ("wavy-2-g3", lambda: si.wavy_cube_mesh(2, 3), 7),
    ("ragged-13x1x1", lambda: si.box_mesh(13, 1, 1, periodic=(True, False, True),
                                           mapping=si.random_affine_mapping(4)), 3),
]


@pytest.mark.parametrize("name,mk,k", CASES, ids=[f"{c[0]}-k{c[2]}" for c in CASES])
def test_mass_block_inverse_matches_oracle(name, mk, k):
    import torch
    hx = _hx()
    print(f"[massinv] {name} k={k}", flush=True)
    p = problem(mk(), k, coef="terrain" if name.startswith("terrain") else "random")
    ctx = gpu_context(p)
    r = si.random_vector(p.n_dofs, 11)
    ref = p.mass_block_apply(r)
    z = ctx.apply_preconditioner(to_dev(r), kind=hx.HX_PC_MASS_BLOCK).cpu().numpy()
    err = np.abs(z - ref).max() / np.abs(ref).max()
    assert err <= 1e-11, (name, k, err)
    z32 = ctx.apply_preconditioner(to_dev(r, torch.float32), kind=hx.HX_PC_MASS_BLOCK)
    err32 = np.abs(z32.cpu().numpy() - ref).max() / np.abs(ref).max()
    assert err32 <= 2e-5, (name, k, err32)
    ctx.close()


def test_pure_mass_problem_one_cg_step():
    """beta = 0 leaves only the mass term (the face terms scale with beta), so
    the exactly inverted mass blocks solve the system in one CG step; the
    step still in flight when convergence is seen must leave x finite."""
    hx = _hx()
    p = problem(si.terrain_mesh(4, 2, 3, g=4), 4, coef="terrain")
    ctx = hx.HelmDG(0)
    ctx.setup_mesh(p.k, p.nodes, p.nbr, p.g)
    ctx.set_coefficients(p.alpha, np.zeros_like(p.beta), p.P)
    b = si.random_vector(p.n_dofs, 5)
    x, info = ctx.solve(to_dev(b), params=hx.default_params(method=0, pc=hx.HX_PC_MASS_BLOCK,
                                                             rtol=1e-11))
    print(f"[massinv] pure mass: {info['iters']} it, res {info['true_rel_res']:.2e}", flush=True)
    assert info["status"] == hx.HX_OK and info["true_rel_res"] <= 1e-11
    assert info["iters"] <= 2
    xs = p.mass_block_apply(b)
    assert np.abs(x.cpu().numpy() - xs).max() <= 1e-11 * np.abs(xs).max()
    ctx.close()


def test_solves_with_mass_block_preconditioner():
    hx = _hx()
    p = problem(si.terrain_mesh(8, 2, 4, g=4), 4, coef="terrain")
    ctx = gpu_context(p)
    b = to_dev(si.rhs_terrain(2)(*p.dof_coords()))
    for method in (0, 1):
        x, info = ctx.solve(b, params=hx.default_params(method=method, pc=hx.HX_PC_MASS_BLOCK,
                                                         rtol=1e-8, max_iter=20000))
        print(f"[massinv] method={method}: {info['iters']} it, {info['ms_total']:.1f} ms, "
              f"res {info['true_rel_res']:.2e}", flush=True)
        assert info["status"] == hx.HX_OK and info["true_rel_res"] <= 1e-8
    x, info = ctx.solve(b, params=hx.default_params(method=1, restart=10, mixed=1,
                                                     pc=hx.HX_PC_MASS_BLOCK, inner_iters=16,
                                                     rtol=1e-8))
    print(f"[massinv] mixed: {info['iters']} outer, {info['inner_iters']} inner", flush=True)
    assert info["status"] == hx.HX_OK and info["true_rel_res"] <= 1e-8
    ctx.close()
