"""The Chebyshev polynomial preconditioner with Lanczos eigenvalue bounds on
the GPU (section 3.1: the technique the paper names for its SPD systems)
against the oracle's recurrence and Lanczos estimate (pinned in
test_chebyshev_oracle.py): the same bounds from the same right-hand side,
the same polynomial applied, and CG with it reaching the true-residual bar
in fewer iterations than with block Jacobi alone."""
import numpy as np
import pytest

import synth_inputs as si
from helpers import gpu_context, problem, to_dev
from oracle.solvers import chebyshev_apply, lanczos_bounds

pytestmark = pytest.mark.gpu


def _hx():
    import paper_2505_00384_amd as hx
    return hx


@pytest.fixture(scope="module")
def terrain():
    p = problem(si.terrain_mesh(8, 2, 4, g=4), 4, coef="terrain")
    return p


def test_lanczos_bounds_match_oracle(terrain):
    p = terrain
    ctx = gpu_context(p)
    b = si.random_vector(p.n_dofs, 31)
    for iters in (5, 20):
        lo, hi = ctx.estimate_eigenvalues(to_dev(b), iters)
        lo_r, hi_r = lanczos_bounds(p.apply, p.bj_apply, b, iters)
        print(f"[cheb] lanczos {iters}: gpu ({lo:.6e}, {hi:.6e}) oracle ({lo_r:.6e}, {hi_r:.6e})",
              flush=True)
        assert abs(lo - lo_r) <= 1e-8 * hi_r and abs(hi - hi_r) <= 1e-8 * hi_r
    ctx.close()


def test_chebyshev_apply_matches_oracle(terrain):
    hx = _hx()
    p = terrain
    ctx = gpu_context(p)
    r = si.random_vector(p.n_dofs, 32)
    for degree, (lo, hi) in ((1, (0.2, 2.5)), (4, (0.05, 1.8)), (7, (0.1, 2.0))):
        ctx.set_chebyshev(degree, lo, hi)
        z = ctx.apply_preconditioner(to_dev(r), kind=hx.HX_PC_CHEBYSHEV).cpu().numpy()
        ref = chebyshev_apply(p.apply, p.bj_apply, r, lo, hi, degree)
        err = np.abs(z - ref).max() / np.abs(ref).max()
        assert err <= 1e-11, (degree, err)
    ctx.close()


def test_cg_with_chebyshev(terrain):
    import torch
    hx = _hx()
    p = terrain
    ctx = gpu_context(p)
    b = to_dev(si.rhs_terrain(4)(*p.dof_coords()))
    g = torch.Generator(device="cuda:0")
    g.manual_seed(3)
    lo, hi = ctx.estimate_eigenvalues(torch.randn(p.n_dofs, dtype=torch.float64, device="cuda:0",
                                                  generator=g), 20)
    _, i_bj = ctx.solve(b, params=hx.default_params(method=0, rtol=1e-8))
    its = {}
    for degree in (2, 4):
        ctx.set_chebyshev(degree, lo, 1.1 * hi)
        x, info = ctx.solve(b, params=hx.default_params(method=0, rtol=1e-8, pc=hx.HX_PC_CHEBYSHEV))
        print(f"[cheb] degree {degree}: {info['iters']} CG iterations ({i_bj['iters']} with block "
              f"Jacobi), {info['ms_total']:.1f} ms vs {i_bj['ms_total']:.1f} ms", flush=True)
        assert info["status"] == hx.HX_OK and info["true_rel_res"] <= 1e-8
        its[degree] = info["iters"]
        _, fi = ctx.solve(b, params=hx.default_params(method=1, rtol=1e-8, pc=hx.HX_PC_CHEBYSHEV))
        assert fi["status"] == hx.HX_OK
    assert its[4] < its[2] < i_bj["iters"]
    ctx.close()


def test_chebyshev_errors(terrain):
    import torch
    hx = _hx()
    p = terrain
    ctx = gpu_context(p)
    b = to_dev(si.rhs_terrain(4)(*p.dof_coords()))
    with pytest.raises(hx.HXError) as e:
        ctx.solve(b, params=hx.default_params(method=0, pc=hx.HX_PC_CHEBYSHEV))
    assert e.value.status == hx.HX_ERR_STATE
    with pytest.raises(hx.HXError) as e:
        ctx.set_chebyshev(3, 1.0, 0.5)
    assert e.value.status == hx.HX_ERR_ARG
    ctx.set_chebyshev(3, 0.1, 2.0)
    with pytest.raises(hx.HXError) as e:
        ctx.solve(b, params=hx.default_params(method=1, mixed=1, pc=hx.HX_PC_CHEBYSHEV))
    assert e.value.status == hx.HX_ERR_ARG
    with pytest.raises(hx.HXError) as e:
        ctx.apply_preconditioner(b.float(), kind=hx.HX_PC_CHEBYSHEV)
    assert e.value.status == hx.HX_ERR_ARG
    ctx.close()
