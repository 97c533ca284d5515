"""The operator with consistent integration (section 3.3: 2k+1 Gauss points
per direction) on the GPU against the oracle's nq-point operator (pinned in
test_overint_oracle.py): the tiny meshes at k = 1, 2, the terrain channel at
k = 4 and curved cells at k = 3, element by element; sampled cells of the
full 256x64x64 channel; and the difference to the fast (k+1)-point operator,
the aliasing the paper trades for speed."""
import numpy as np
import pytest

import synth_inputs as si
from helpers import TINY, gpu_context, normwise, problem, to_dev

pytestmark = pytest.mark.gpu

CASES = [(name, mk, k) for (name, mk) in TINY for k in (1, 2)] + [
    ("terrain-4x2x3-g4", lambda: si.terrain_mesh(4, 2, 3, g=4), 4),
    ("wavy-2-g3", lambda: si.wavy_cube_mesh(2, 3), 3),
    ("terrain-2x1x2-g4", lambda: si.terrain_mesh(2, 1, 2, g=4), 6),
]


@pytest.mark.parametrize("name,mk,k", CASES, ids=[f"{c[0]}-k{c[2]}" for c in CASES])
def test_consistent_operator_matches_oracle(name, mk, k):
    print(f"[consistent] {name} k={k}", flush=True)
    p = problem(mk(), k, coef="terrain" if name.startswith("terrain") else "random")
    ctx = gpu_context(p)
    ctx.set_consistent(p.alpha, p.beta)
    x = si.random_vector(p.n_dofs, 17)
    y = ctx.apply_consistent(to_dev(x)).cpu().numpy()
    ref = p.apply_q(x, 2 * k + 1)
    e2, einf = normwise(y, ref)
    assert e2 <= 1e-12 and einf <= 1e-12, (name, k, e2, einf)
    # the fast operator differs from it by the aliasing of the (k+1)-point rule
    yf = ctx.apply_operator(to_dev(x)).cpu().numpy()
    np.testing.assert_allclose(normwise(yf, ref)[0], normwise(p.apply(x), ref)[0], rtol=1e-6,
                               atol=1e-14)
    ctx.close()


def test_consistent_sampled_full_size():
    import torch
    free = torch.cuda.mem_get_info()[0]
    if free < 120e9:
        pytest.skip("needs ~120 GB of device memory")
    print("[consistent] terrain 256x64x64 k=4, sampled cells", flush=True)
    m = si.terrain_mesh(256, 64, 64, g=4)
    p = problem(m, 4, coef="terrain")
    ctx = gpu_context(p)
    ctx.set_consistent(p.alpha, p.beta)
    x = si.random_vector(p.n_dofs, 5)
    y = ctx.apply_consistent(to_dev(x)).cpu().numpy().reshape(m.n_cells, -1)
    rng = np.random.default_rng(0)
    cells = np.unique(np.concatenate([rng.integers(0, m.n_cells, 16),
                                      [0, 255, 256 * 63, m.n_cells - 1]]))
    ref = p.apply_q_cells(x, cells, 9)
    e2, einf = normwise(y[cells], ref)
    assert e2 <= 1e-12 and einf <= 1e-12, (e2, einf)
    ctx.close()


def _oracle_cg(p, apply, b, precond, rtol):
    from oracle import solvers
    return solvers.cg(apply, b, precond=precond, rtol=rtol, max_iter=2000)


def test_consistent_system_solve_matches_oracle():
    """CG on the consistently integrated operator (system 2) preconditioned by
    the fast-form block Jacobi: the oracle's CG with its nq-point operator
    and separable block takes the same iterations (within one), and the
    solutions agree with the oracle's tight solve."""
    hx = __import__("paper_2505_00384_amd")
    p = problem(si.terrain_mesh(8, 2, 4, g=4), 4, coef="terrain")
    ctx = gpu_context(p)
    ctx.set_consistent(p.alpha, p.beta)
    b = p.load_vector(si.rhs_terrain(2))
    apply_q = lambda v: p.apply_q(v, 9)
    x_ref, i_ref = _oracle_cg(p, apply_q, b, p.bj_apply, 1e-8)
    x_tight, _ = _oracle_cg(p, apply_q, b, p.bj_apply, 1e-13)
    x, info = ctx.solve(to_dev(b), params=hx.default_params(method=0, rtol=1e-8, system=2))
    print(f"[consistent] CG system 2: {info['iters']} iterations (oracle {i_ref.iters})",
          flush=True)
    assert info["status"] == hx.HX_OK and info["true_rel_res"] <= 1e-8
    assert abs(info["iters"] - i_ref.iters) <= 1
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs - x_tight) <= 1e-6 * np.linalg.norm(x_tight)
    # the oracle's residual of the GPU solution, with the oracle's operator
    assert np.linalg.norm(b - apply_q(xs)) <= 1.01e-8 * np.linalg.norm(b)
    # FGMRES on the same system
    x2, i2 = ctx.solve(to_dev(b), params=hx.default_params(method=1, rtol=1e-8, system=2))
    assert i2["status"] == hx.HX_OK and i2["true_rel_res"] <= 1e-8
    # the fast system differs from the consistent one by the aliasing
    xf, _ = ctx.solve(to_dev(b), params=hx.default_params(method=0, rtol=1e-10))
    d = float((xf - x).norm() / x.norm())
    print(f"[consistent] fast vs consistent solution: {d:.2e}", flush=True)
    assert 1e-9 < d < 1e-2
    ctx.close()


def test_consistent_weighted_mass_solve():
    """The alpha-weighted mass with 2k+1 points (beta = 0) solved by CG with the
    fast (k+1)-point mass-block inverse as preconditioner: the paper's
    consistent treatment of its modified mass matrix against its fast direct
    inverse; the oracle's CG with its mass-block solve takes the same
    iterations, and the solutions agree."""
    hx = __import__("paper_2505_00384_amd")
    p = problem(si.terrain_mesh(4, 2, 3, g=4), 4, coef="terrain")
    ctx = gpu_context(p)
    zero = np.zeros(p.n_dofs)
    ctx.set_consistent(p.alpha, zero)
    import oracle
    pm = oracle.Problem(p.mesh, 4, p.alpha, zero)
    b = si.random_vector(p.n_dofs, 3)
    apply_q = lambda v: pm.apply_q(v, 9)
    x_ref, i_ref = _oracle_cg(pm, apply_q, b, pm.mass_block_apply, 1e-12)
    x, info = ctx.solve(to_dev(b), params=hx.default_params(method=0, rtol=1e-12, system=2,
                                                            pc=hx.HX_PC_MASS_BLOCK))
    print(f"[consistent] weighted mass: {info['iters']} CG iterations (oracle {i_ref.iters})",
          flush=True)
    assert info["status"] == hx.HX_OK and info["true_rel_res"] <= 1e-12
    assert abs(info["iters"] - i_ref.iters) <= 1 and info["iters"] <= 12
    assert np.abs(x.cpu().numpy() - x_ref).max() <= 1e-10 * np.abs(x_ref).max()
    # the fast inverse alone solves the (k+1)-point mass exactly, the
    # consistent mass only up to the aliasing of the weight
    z = ctx.apply_preconditioner(to_dev(b), kind=hx.HX_PC_MASS_BLOCK).cpu().numpy()
    d = np.linalg.norm(z - x_ref) / np.linalg.norm(x_ref)
    print(f"[consistent] fast inverse vs consistent mass solve: {d:.2e}", flush=True)
    assert 1e-12 < d < 1e-1
    ctx.close()


def test_consistent_system_with_multigrid():
    """The consistent system preconditioned by the fast operator's V-cycle
    (three levels): converges to the bar in at most twice the iterations of
    the fast system with the same cycle."""
    hx = __import__("paper_2505_00384_amd")
    from helpers import terrain_hierarchy, oracle_levels
    probs, maps = terrain_hierarchy(16, 4, 8, 3, 3)
    levels = oracle_levels(probs, maps)
    ctxs = [gpu_context(L.prob) for L in levels]
    for l, L in enumerate(levels):
        ctxs[l].set_chebyshev(L.degree, L.lo, L.hi)
        if l + 1 < len(levels):
            ctxs[l].set_multigrid(ctxs[l + 1], L.parent, L.octant)
    p = probs[0]
    ctxs[0].set_consistent(p.alpha, p.beta)
    b = to_dev(p.load_vector(si.rhs_terrain(0)))
    _, i_fast = ctxs[0].solve(b, params=hx.default_params(method=0, rtol=1e-8,
                                                          pc=hx.HX_PC_MULTIGRID_MIXED))
    _, i_q = ctxs[0].solve(b, params=hx.default_params(method=0, rtol=1e-8, system=2,
                                                       pc=hx.HX_PC_MULTIGRID_MIXED))
    print(f"[consistent] CG + V-cycle: fast system {i_fast['iters']}, consistent system "
          f"{i_q['iters']} iterations", flush=True)
    assert i_q["status"] == hx.HX_OK and i_q["true_rel_res"] <= 1e-8
    assert i_q["iters"] <= 2 * i_fast["iters"]
    for c in ctxs:
        c.close()
