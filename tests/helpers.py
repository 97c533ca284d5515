"""Shared set-up for the GPU parity tests: one seeded input, given to both the
HIP library and the oracle."""
import numpy as np

import oracle
import synth_inputs as si


def problem(mesh, k, coef="random", seed=0, P=2.0):
    """Oracle problem with coefficient fields evaluated at the oracle's own dof
    coordinates; the same arrays are then handed to the library."""
    p = oracle.Problem(mesh, k, P=P)
    if coef == "terrain":
        fa, fb = si.terrain_coefficients()
    elif coef == "const":
        fa, fb = si.const_coefficients(1.0, 0.01)
    else:
        fa, fb = si.random_smooth_coefficients(seed)
    p.set_coefficient_functions(fa, fb)
    return p


def gpu_context(p):
    import paper_2505_00384_amd as hx
    ctx = hx.HelmDG(0)
    ctx.setup_mesh(p.k, p.nodes, p.nbr, p.g, hang=p.hang if p.hang.shape[0] else None)
    ctx.set_coefficients(p.alpha, p.beta, p.P)
    return ctx


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def normwise(y, ref):
    """(||y - ref||_2 / ||ref||_2, max|y - ref| / max|ref|)"""
    d = np.asarray(y, dtype=np.float64) - ref
    return (np.linalg.norm(d) / np.linalg.norm(ref), np.abs(d).max() / np.abs(ref).max())


TINY = [
    ("1x1x1-periodic", lambda: si.box_mesh(1, 1, 1, periodic=(True, True, True))),
    ("2x1x3-periodic", lambda: si.box_mesh(2, 1, 3, periodic=(True, True, True))),
    ("3x3x3-neumann", lambda: si.cube_mesh(3, periodic=(False, False, False))),
    ("terrain-3x2x2-g2", lambda: si.terrain_mesh(3, 2, 2, g=2)),
    ("wavy-3-g3", lambda: si.wavy_cube_mesh(3, 3)),
    ("jitter-3x2x2", lambda: si.random_node_jitter(
        si.box_mesh(3, 2, 2, periodic=(False,) * 3, g=2), 4, 0.03)),
    ("ragged-7x1x1", lambda: si.box_mesh(7, 1, 1, periodic=(True, False, True),
                                          mapping=si.random_affine_mapping(9))),
]


def oracle_fixed_point(mesh, k, rho, F, G, p0, gamma, tau, iters):
    """The fixed point of the pressure system, step by step in the oracle:
    h from the previous iterate (ideal gas, h = gamma p / ((gamma - 1) rho)),
    rebuild the system, solve it tightly (FGMRES, inverse Helmholtz diagonal)."""
    from oracle.core import PressureSystem
    p = np.array(p0, dtype=np.float64)
    for _ in range(iters):
        h = gamma * p / ((gamma - 1.0) * rho)
        ref = PressureSystem(mesh, k, rho, h, gamma, tau)
        helm = oracle.Problem(mesh, k, alpha=np.full(p.size, 1.0 / (gamma - 1.0)),
                              beta=tau ** 2 * h)
        dinv = 1.0 / helm.cell_diagonal(stiff=True)
        p, info = oracle.solvers.fgmres(ref.apply, ref.rhs(F, G), precond=lambda v: dinv * v,
                                        restart=30, rtol=1e-13, max_iter=5000, x0=p)
        assert info.converged
    return p


def constructed_pressure_state(mesh, k, gamma):
    """A perturbed hydrostatic pressure p* on the terrain channel and data
    (rho, F, G) for which p* is the fixed point: G = S(h(p*)) p* + C A^-1 F.
    Returns rho, F, G, p_background, p_star, tau."""
    from oracle.core import PressureSystem
    p_or = oracle.Problem(mesh, k)
    x, y, z = p_or.dof_coords()
    T = si.TERRAIN
    rho = np.exp(-z / T["H"])
    p_bg = 1e5 * np.exp(-z / T["H"])
    p_star = p_bg * (1.0 + 0.02 * np.sin(2 * np.pi * x / T["Lx"]) * np.cos(np.pi * z / T["Lz"]))
    F = 10.0 * rho * np.stack([si.rhs_terrain(s)(x, y, z) for s in (41, 42, 43)])
    tau = T["dt"]
    ref = PressureSystem(mesh, k, rho, gamma * p_star / ((gamma - 1.0) * rho), gamma, tau)
    G = ref.apply(p_star) + ref.div(ref.a_inv(F))
    return rho, F, G, p_bg, p_star, tau


def terrain_hierarchy(nx, ny, nz, n_levels, k, g=None):
    """Terrain channels (nx, ny, nz), (nx/2, ny/2, nz/2), ... with the terrain
    coefficients at each level's own dofs, and the cell maps between them."""
    probs, maps = [], []
    for l in range(n_levels):
        s = 2 ** l
        m = si.terrain_mesh(nx // s, ny // s, nz // s, g=k if g is None else g)
        probs.append(problem(m, k, coef="terrain"))
        if l + 1 < n_levels:
            maps.append(si.refinement_parents(nx // (2 * s), ny // (2 * s), nz // (2 * s)))
    return probs, maps


def oracle_levels(probs, maps, smooth_degree=3, smooth_ratio=15.0, coarse_degree=12,
                  lanczos_iters=20):
    """Oracle multigrid levels: Chebyshev smoothing on [1.1 hi / ratio, 1.1 hi]
    of each level's estimated range, the coarsest level's polynomial on
    [0.9 lo, 1.1 hi]; the estimates come from the oracle's Lanczos process."""
    from oracle.multigrid import Level
    from oracle import solvers
    levels = []
    for l, p in enumerate(probs):
        b = si.random_vector(p.n_dofs, 100 + l)
        lo, hi = solvers.lanczos_bounds(p.apply, p.bj_apply, b, lanczos_iters)
        if l + 1 < len(probs):
            levels.append(Level(p, smooth_degree, 1.1 * hi / smooth_ratio, 1.1 * hi, *maps[l]))
        else:
            levels.append(Level(p, coarse_degree, 0.9 * lo, 1.1 * hi))
    return levels
