"""The paper's diagonal preconditioners on the GPU (section 3.1): the
"Helmholtz preconditioner", the inverse diagonal of the volume terms of the
form, and its "internal-energy" variant, the inverse mass diagonal.  The
diagonals formed by hx_set_coefficients from the merged cell data are compared
with the oracle's direct-quadrature diagonals (pinned in
test_diag_oracle.py); the preconditioners are applied in FP64 and FP32, and
CG and FGMRES reach the true-residual bar with them."""
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
]


@pytest.mark.parametrize("name,mk,k", CASES, ids=[f"{c[0]}-k{c[2]}" for c in CASES])
def test_diagonals_match_oracle(name, mk, k):
    hx = _hx()
    print(f"[diag] {name} k={k}", flush=True)
    p = problem(mk(), k, coef="terrain" if name.startswith("terrain") else "random")
    ctx = gpu_context(p)
    inv = ctx.debug_export(hx.HX_EXPORT_INV_DIAG, (2, p.n_dofs))
    for row, stiff in ((0, True), (1, False)):
        ref = p.cell_diagonal(stiff=stiff)
        got = 1.0 / inv[row]
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err <= 1e-12, (name, k, stiff, err)
    ctx.close()


def test_apply_fp64_fp32():
    import torch
    hx = _hx()
    p = problem(si.terrain_mesh(4, 2, 3, g=4), 4, coef="terrain")
    ctx = gpu_context(p)
    r = si.random_vector(p.n_dofs, 3)
    for kind, stiff in ((hx.HX_PC_HELMHOLTZ_DIAG, True), (hx.HX_PC_MASS_DIAG, False)):
        ref = r / p.cell_diagonal(stiff=stiff)
        z = ctx.apply_preconditioner(to_dev(r), kind=kind).cpu().numpy()
        assert np.abs(z - ref).max() <= 1e-13 * np.abs(ref).max()
        z32 = ctx.apply_preconditioner(to_dev(r, torch.float32), kind=kind).cpu().numpy()
        assert np.abs(z32 - ref).max() <= 1e-6 * np.abs(ref).max()
    ctx.close()


def test_solves_with_diagonal_preconditioners():
    hx = _hx()
    p = problem(si.terrain_mesh(8, 2, 4, g=4), 4, coef="terrain")
    ctx = gpu_context(p)
    b = to_dev(si.rhs_terrain(2)(*p.dof_coords()))
    its = {}
    for name, kind in (("helmholtz", hx.HX_PC_HELMHOLTZ_DIAG), ("mass", hx.HX_PC_MASS_DIAG),
                       ("bj", hx.HX_PC_BLOCK_JACOBI)):
        for method in (0, 1):
            x, info = ctx.solve(b, params=hx.default_params(method=method, pc=kind, rtol=1e-8,
                                                             max_iter=20000))
            print(f"[diag] {name} method={method}: {info['iters']} it, "
                  f"{info['ms_total']:.1f} ms, res {info['true_rel_res']:.2e}", flush=True)
            assert info["status"] == hx.HX_OK and info["true_rel_res"] <= 1e-8
            its[(name, method)] = info["iters"]
    # the volume diagonal is the better diagonal; the block preconditioner beats both
    assert its[("helmholtz", 0)] < its[("mass", 0)]
    assert its[("bj", 0)] < its[("helmholtz", 0)]
    ctx.close()


def test_mixed_solve_with_diagonal_inner_preconditioner():
    """The inner FP32 CG of the mixed form takes the chosen kind; the learned
    kind (FP64 only) is refused there."""
    hx = _hx()
    p = problem(si.terrain_mesh(8, 2, 4, g=4), 4, coef="terrain")
    ctx = gpu_context(p)
    b = to_dev(si.rhs_terrain(5)(*p.dof_coords()))
    for kind in (hx.HX_PC_HELMHOLTZ_DIAG, hx.HX_PC_BLOCK_JACOBI):
        x, info = ctx.solve(b, params=hx.default_params(method=1, restart=10, mixed=1, pc=kind,
                                                         inner_iters=16, rtol=1e-8))
        print(f"[diag] mixed inner pc={kind}: {info['iters']} outer, {info['inner_iters']} inner",
              flush=True)
        assert info["status"] == hx.HX_OK and info["true_rel_res"] <= 1e-8
    with pytest.raises(hx.HXError):
        ctx.solve(b, params=hx.default_params(method=1, mixed=1, pc=hx.HX_PC_LEARNED))
    ctx.close()
