"""Pins of the CPU oracle against facts it does not compute itself.

Each test fixes the oracle to something other than its own code: closed forms
of the Gauss rules, library routines (numpy's Gauss-Legendre), the paper's
construction of a matrix-free operator's matrix by unit vectors (section 3.1)
against an independent element/face assembly, a Kronecker closed form built
here from 1-D matrices, invariants (symmetry, positivity, constants), exact
reproduction of polynomials and manufactured-solution convergence rates.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth_inputs as si

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold_rules():
    out = {}
    for line in open(os.path.join(GOLD, "gauss_rules.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, kind, x, w = line.split()
        out.setdefault((int(n), kind), []).append((float(x), float(w)))
    return out


def _gold_const(name):
    for line in open(os.path.join(GOLD, "constants.txt")):
        if line.startswith(name + " "):
            return float(line.split()[1])
    raise KeyError(name)


# ---------------------------------------------------------------------------
# 1-D rules and basis
# ---------------------------------------------------------------------------

def test_rules_match_closed_forms():
    gold = _gold_rules()
    for (n, kind), vals in gold.items():
        x, w = (oracle.gauss_legendre if kind == "GL" else oracle.gauss_lobatto)(n)
        gx = np.array([v[0] for v in vals]); gw = np.array([v[1] for v in vals])
        np.testing.assert_allclose(2 * x - 1, gx, atol=1e-15)
        np.testing.assert_allclose(2 * w, gw, atol=1e-15)


@pytest.mark.parametrize("n", range(2, 10))
def test_rules_exactness_and_library(n):
    x, w = oracle.gauss_legendre(n)
    xl, wl = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(2 * x - 1, xl, atol=2e-15)
    np.testing.assert_allclose(2 * w, wl, atol=2e-15)
    for p in range(2 * n):                     # GL exact to degree 2n-1
        assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 5e-15
    x, w = oracle.gauss_lobatto(n)
    for p in range(2 * n - 2):                 # GLL exact to degree 2n-3
        assert abs(np.sum(w * x ** p) - 1.0 / (p + 1)) < 5e-15
    # GLL interior nodes are the roots of P'_{n-1}
    if n > 2:
        roots = np.sort(np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots())
        np.testing.assert_allclose(2 * x[1:-1] - 1, roots, atol=1e-14)
    # not exact at degree 2n-2 (a rule with n nodes cannot be)
    assert abs(np.sum(w * x ** (2 * n - 2)) - 1.0 / (2 * n - 1)) > 1e-12


@pytest.mark.parametrize("n", [2, 3, 5, 7])
def test_lagrange_basis(n):
    nodes, _ = oracle.gauss_lobatto(n)
    for j, t in enumerate(nodes):
        v, _ = oracle.lagrange(nodes, t)
        np.testing.assert_allclose(v, np.eye(n)[j], atol=1e-14)
    rng = np.random.default_rng(0)
    coef = rng.normal(size=n)
    for t in rng.uniform(0, 1, 7):
        v, d = oracle.lagrange(nodes, t)
        assert abs(v.sum() - 1) < 1e-13 and abs(d.sum()) < 1e-11
        # exact interpolation and derivative of a degree n-1 polynomial
        pv = np.polyval(coef, nodes)
        assert abs(v @ pv - np.polyval(coef, t)) < 1e-12
        assert abs(d @ pv - np.polyval(np.polyder(coef), t)) < 1e-10


# ---------------------------------------------------------------------------
# the operator's matrix: unit vectors (section 3.1) == element/face assembly
# ---------------------------------------------------------------------------

def _tiny_meshes():
    return [
        ("1x1x1-periodic", si.box_mesh(1, 1, 1, periodic=(True, True, True))),
        ("2x2x2-periodic", si.cube_mesh(2)),
        ("2x1x3-periodic", si.box_mesh(2, 1, 3, periodic=(True, True, True))),
        ("2x2x2-neumann", si.cube_mesh(2, periodic=(False, False, False))),
        ("terrain-2x1x2", si.terrain_mesh(2, 1, 2, g=2)),
        ("wavy-2", si.wavy_cube_mesh(2, 2)),
        ("sheared-2", si.box_mesh(2, 2, 1, periodic=(False, True, False),
                                  mapping=si.random_affine_mapping(5))),
    ]


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_unit_vector_matrix_equals_assembly(k):
    for name, m in _tiny_meshes():
        if k == 4 and m.n_cells > 4:
            continue
        p = oracle.Problem(m, k)
        fa, fb = si.random_smooth_coefficients(k)
        if name.startswith("terrain"):
            fa, fb = si.terrain_coefficients()
        p.set_coefficient_functions(fa, fb)
        A1 = p.matrix_by_unit_vectors()
        A2 = p.assemble_dense()
        scale = np.abs(A2).max()
        assert np.abs(A1 - A2).max() <= 1e-13 * scale, name
        # symmetry and positivity
        assert np.abs(A2 - A2.T).max() <= 1e-14 * scale, name
        assert np.linalg.eigvalsh(0.5 * (A2 + A2.T)).min() > 0, name


# ---------------------------------------------------------------------------
# Cartesian closed form: A = a h^3 M(x)M(x)M + b h (L(x)M(x)M + ...)
# built here from 1-D matrices with numpy's own rules
# ---------------------------------------------------------------------------

def _np_rules(n):
    xq, wq = np.polynomial.legendre.leggauss(n)
    xq, wq = 0.5 * (xq + 1), 0.5 * wq
    r = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots() if n > 2 else np.array([])
    xl = np.concatenate([[0.0], 0.5 * (np.sort(r) + 1), [1.0]])
    return xq, wq, xl


def _np_lagrange(xl, t):
    """values and derivatives of the Lagrange basis at t (numpy polyfit-free)."""
    n = xl.size
    V = np.vander(xl, n, increasing=True)
    C = np.linalg.inv(V)           # column i: monomial coefficients of l_i
    pw = np.array([t ** m for m in range(n)])
    dpw = np.array([m * t ** (m - 1) if m > 0 else 0.0 for m in range(n)])
    return pw @ C, dpw @ C


def _sip_1d(nc, k, pen, periodic):
    n = k + 1
    xq, wq, xl = _np_rules(n)
    Mh = np.zeros((n, n)); L0 = np.zeros((n, n))
    for x, w in zip(xq, wq):
        v, d = _np_lagrange(xl, x)
        Mh += w * np.outer(v, v); L0 += w * np.outer(d, d)
    v0, d0 = _np_lagrange(xl, 0.0)
    v1, d1 = _np_lagrange(xl, 1.0)
    N = nc * n
    M = np.zeros((N, N)); L = np.zeros((N, N))
    for c in range(nc):
        s = slice(c * n, (c + 1) * n)
        M[s, s] = Mh; L[s, s] += L0
    for c in range(nc):                      # face at the right end of cell c
        cp = c + 1
        if cp == nc:
            if not periodic:
                continue
            cp = 0
        # side values/derivatives: minus = cell c at 1, plus = cell cp at 0
        side = {0: (c, v1, d1, 1.0), 1: (cp, v0, d0, -1.0)}
        for st in (0, 1):
            ct, vt, dt, zt = side[st]
            for su in (0, 1):
                cu, vu, du, zu = side[su]
                blk = (-0.5 * np.outer(zt * vt, du) - 0.5 * np.outer(dt, zu * vu)
                       + pen * np.outer(zt * vt, zu * vu))
                L[ct * n:(ct + 1) * n, cu * n:(cu + 1) * n] += blk
    return M, L


@pytest.mark.parametrize("k,nc,periodic", [(2, 4, True), (1, 3, True), (3, 2, False), (4, 2, True)])
def test_cartesian_kronecker_closed_form(k, nc, periodic):
    alpha, beta, P = 1.3, 0.01 * nc * nc * 2.0, 2.0
    h = 1.0 / nc
    m = si.cube_mesh(nc, periodic=(periodic,) * 3)
    p = oracle.Problem(m, k, P=P)
    p.set_coefficient_functions(*si.const_coefficients(alpha, beta))
    n = k + 1
    pen = P * n * n  # sigma_F h = P (k+1)^2 |F| h / |K| = P (k+1)^2
    M, L = _sip_1d(nc, k, pen, periodic)
    A_k = alpha * h ** 3 * np.kron(M, np.kron(M, M)) + beta * h * (
        np.kron(M, np.kron(M, L)) + np.kron(M, np.kron(L, M)) + np.kron(L, np.kron(M, M)))
    # permutation from Kronecker order (x fastest, global 1-D indices) to cells
    N1 = nc * n
    perm = np.empty(p.n_dofs, dtype=np.int64)
    for cz in range(nc):
        for cy in range(nc):
            for cx in range(nc):
                cell = cx + nc * (cy + nc * cz)
                for l in range(n):
                    for j in range(n):
                        for i in range(n):
                            I = (cx * n + i) + N1 * ((cy * n + j) + N1 * (cz * n + l))
                            perm[cell * n ** 3 + i + n * (j + n * l)] = I
    A_ref = A_k[np.ix_(perm, perm)]
    A = p.assemble_dense()
    assert np.abs(A - A_ref).max() <= 1e-13 * np.abs(A_ref).max()
    # the face penalty of this mesh is the closed form 2 (k+1)^2 / h
    s = p.face_sigma()
    if periodic:
        np.testing.assert_allclose(s, P * n * n / h, rtol=1e-13)


def test_penalty_golden():
    m = si.cube_mesh(4)
    p = oracle.Problem(m, 2)
    np.testing.assert_allclose(p.face_sigma(), _gold_const("penalty_cube4_k2"), rtol=1e-13)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def test_constants_and_volumes():
    # A 1 depends only on alpha (no gradient, no jump), on every mesh
    for name, m in _tiny_meshes():
        p = oracle.Problem(m, 2)
        fa, fb = si.random_smooth_coefficients(1)
        p.set_coefficient_functions(fa, fb)
        y1 = p.apply(np.ones(p.n_dofs))
        p.set_coefficient_functions(fa, lambda x, y, z: 7.0 * fb(x, y, z) + 1.0)
        y2 = p.apply(np.ones(p.n_dofs))
        assert np.abs(y1 - y2).max() <= 1e-13 * np.abs(y1).max(), name
    # sum(A 1) with alpha = 1 is the volume
    m = si.cube_mesh(3)
    p = oracle.Problem(m, 3); p.set_coefficient_functions(*si.const_coefficients(1.0, 0.2))
    assert abs(p.apply(np.ones(p.n_dofs)).sum() - 1.0) < 1e-13
    f = si.random_affine_mapping(2)
    A = np.array([f(*e) for e in np.eye(3)]).T
    m = si.box_mesh(2, 2, 2, periodic=(False,) * 3, mapping=f)
    p = oracle.Problem(m, 2); p.set_coefficient_functions(*si.const_coefficients(1.0, 0.2))
    assert abs(p.apply(np.ones(p.n_dofs)).sum() - abs(np.linalg.det(A))) < 1e-13
    # terrain channel volume converges to the closed form
    V = _gold_const("terrain_volume")
    errs = []
    for nx in (4, 8, 16, 32):
        m = si.terrain_mesh(nx, 1, 1, g=4)
        p = oracle.Problem(m, 4)
        errs.append(abs(p.cell_volumes().sum() - V) / V)
    assert errs[-1] < 1e-12 and errs[3] < errs[2] < errs[1] < errs[0]


def _quad_err(p, u, fexact):
    xyz, w = p.quad_data()
    uq = np.zeros(p.n_dofs)
    oracle.core.lib().or_eval_quad(p._s(), oracle.core._dp(np.ascontiguousarray(u)), oracle.core._dp(uq))
    return math.sqrt(np.sum(w * (uq - fexact(*xyz)) ** 2))


def test_polynomial_reproduction_neumann_cube():
    """A I(p) = int (a p - b lap p) phi + int_{bdry} b dn p phi for p in Q_k:
    every integrand is exact with (k+1)-point Gauss, so equality is exact.
    The right side is computed here from 1-D integrals (p separable)."""
    rng = np.random.default_rng(1)
    for k in (1, 2, 3, 4):
        nc = 2
        n = k + 1
        alpha, beta = 0.7, 0.3
        m = si.cube_mesh(nc, periodic=(False,) * 3)
        p = oracle.Problem(m, k)
        p.set_coefficient_functions(*si.const_coefficients(alpha, beta))
        cs = [rng.normal(size=k + 1) for _ in range(3)]     # 1-D factors
        q = [np.polynomial.Polynomial(c) for c in cs]
        xyz = p.dof_coords()
        u = q[0](xyz[0]) * q[1](xyz[1]) * q[2](xyz[2])
        Au = p.apply(u)
        # rhs from 1-D integrals over each cell, reference basis on GLL nodes
        xq, wq, xl = _np_rules(n)
        h = 1.0 / nc
        b = np.zeros(p.n_dofs)
        for cell in range(m.n_cells):
            cidx = (cell % nc, (cell // nc) % nc, cell // (nc * nc))
            I = []   # per direction: int f phi_i for f in (q, q'')
            for d in range(3):
                a0 = cidx[d] * h
                i0 = np.zeros(n); i2 = np.zeros(n)
                for x, w in zip(xq, wq):
                    v, _ = _np_lagrange(xl, x)
                    X = a0 + h * x
                    i0 += w * h * q[d](X) * v
                    i2 += w * h * q[d].deriv(2)(X) * v
                I.append((i0, i2))
            loc = np.zeros((n, n, n))
            for l in range(n):
                for j in range(n):
                    for i in range(n):
                        val = alpha * I[0][0][i] * I[1][0][j] * I[2][0][l]
                        lap = (I[0][1][i] * I[1][0][j] * I[2][0][l] + I[0][0][i] * I[1][1][j] * I[2][0][l]
                               + I[0][0][i] * I[1][0][j] * I[2][1][l])
                        loc[l, j, i] = val - beta * lap
            # boundary: int b dn p phi over faces on the domain boundary
            for d in range(3):
                for end in (0, 1):
                    if cidx[d] != (0 if end == 0 else nc - 1):
                        continue
                    X = float(end)
                    dn = (1.0 if end else -1.0) * q[d].deriv(1)(X)
                    li = 0 if end == 0 else n - 1
                    others = [e for e in range(3) if e != d]
                    for a in range(n):
                        for c2 in range(n):
                            idx = [0, 0, 0]
                            idx[d] = li; idx[others[0]] = a; idx[others[1]] = c2
                            loc[idx[2], idx[1], idx[0]] += beta * dn * I[others[0]][0][a] * I[others[1]][0][c2] \
                                / (q[others[0]](0) * 0 + 1)
            b[cell * n ** 3:(cell + 1) * n ** 3] = loc.ravel()
        assert np.abs(Au - b).max() <= 1e-12 * np.abs(b).max(), k


@pytest.mark.slow
@pytest.mark.parametrize("k,sizes,mesh", [(2, (2, 4, 8), "cube"), (4, (1, 2, 4), "cube"),
                                          (2, (2, 4, 8), "wavy")])
def test_manufactured_solution_rates(k, sizes, mesh):
    tp = 2 * math.pi
    alpha, beta = 1.0, 0.05

    def uex(x, y, z):
        return np.sin(tp * x) * np.cos(tp * y) * np.sin(tp * z + 0.3)

    def f(x, y, z):
        return (alpha + beta * 3 * tp * tp) * uex(x, y, z)
    errs = []
    for nc in sizes:
        m = si.cube_mesh(nc, g=1) if mesh == "cube" else si.wavy_cube_mesh(nc, g=k, eps=0.03)
        p = oracle.Problem(m, k)
        p.set_coefficient_functions(*si.const_coefficients(alpha, beta))
        b = p.load_vector(f)
        x, info = oracle.solvers.cg(p.apply, b, precond=p.bj_apply, rtol=1e-12, max_iter=2000)
        assert info.converged
        errs.append(_quad_err(p, x, uex))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert rates[-1] > k + 1 - 0.35, (errs, rates)


# ---------------------------------------------------------------------------
# separable cell block
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("k", [1, 2, 4])
def test_bj_sep_equals_exact_block_on_cartesian(k):
    m = si.box_mesh(3, 3, 3, periodic=(True, False, True), lo=(0, 0, 0), hi=(1.5, 0.9, 0.6))
    p = oracle.Problem(m, k)
    p.set_coefficient_functions(*si.const_coefficients(0.8, 0.05))
    A = p.assemble_dense()
    nd = (k + 1) ** 3
    for c in (0, 4, 13, 26):
        blk = A[c * nd:(c + 1) * nd, c * nd:(c + 1) * nd]
        Ab = p.bj_sep_block(c)
        assert np.abs(blk - Ab).max() <= 1e-13 * np.abs(blk).max()
    r = si.random_vector(p.n_dofs, 3)
    z = p.bj_apply(r)
    for c in range(m.n_cells):
        blk = A[c * nd:(c + 1) * nd, c * nd:(c + 1) * nd]
        np.testing.assert_allclose(blk @ z[c * nd:(c + 1) * nd], r[c * nd:(c + 1) * nd],
                                   rtol=1e-10, atol=1e-10 * np.abs(r).max())


def test_bj_sep_spd_on_curved_cells():
    m = si.terrain_mesh(4, 2, 2, g=4)
    p = oracle.Problem(m, 4)
    p.set_coefficient_functions(*si.terrain_coefficients())
    for c in range(m.n_cells):
        Ab = p.bj_sep_block(c)
        assert np.abs(Ab - Ab.T).max() <= 1e-14 * np.abs(Ab).max()
        assert np.linalg.eigvalsh(Ab).min() > 0


# ---------------------------------------------------------------------------
# solvers
# ---------------------------------------------------------------------------

def test_cg_and_fgmres_match_dense_solve():
    m = si.cube_mesh(4)
    p = oracle.Problem(m, 2)
    p.set_coefficient_functions(*si.const_coefficients(1.0, 0.01))
    A = p.assemble_dense()
    xyz = p.dof_coords()
    b = si.rhs_cube(0)(*xyz)
    xs = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A)
    x, info = oracle.solvers.cg(p.apply, b, precond=p.bj_apply, rtol=1e-10)
    assert info.converged and info.true_rel_res <= 1e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-10
    x2, info2 = oracle.solvers.fgmres(p.apply, b, precond=p.bj_apply, restart=30, rtol=1e-10)
    assert info2.converged
    assert np.linalg.norm(x2 - xs) / np.linalg.norm(xs) <= kappa * 1e-10
    # unpreconditioned CG takes more iterations than block-Jacobi CG
    _, info3 = oracle.solvers.cg(p.apply, b, precond=None, rtol=1e-10)
    assert info3.iters > info.iters


def test_fgmres_fallback_policy():
    m = si.cube_mesh(2)
    p = oracle.Problem(m, 2)
    p.set_coefficient_functions(*si.const_coefficients(1.0, 0.05))
    b = si.random_vector(p.n_dofs, 1)
    bad = lambda v: v * np.nan
    x, info = oracle.solvers.fgmres(p.apply, b, precond=bad, fallback=p.bj_apply, rtol=1e-9)
    assert info.fallback_used and info.converged
    e0 = np.zeros(p.n_dofs); e0[0] = 1.0
    const = lambda v: e0.copy()         # the Krylov space stops growing: stagnation
    x, info = oracle.solvers.fgmres(p.apply, b, precond=const, fallback=p.bj_apply, rtol=1e-9,
                                    restart=30)
    assert info.fallback_used and info.converged
