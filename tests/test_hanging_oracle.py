"""Pins of the oracle on non-conforming meshes (2:1 hanging faces).

The paper's second mesh refines part of the domain, so a coarse cell meets
four finer ones across a face.  Each quarter of such a face carries the same
interior-penalty terms, integrated with the fine face's Gauss rule, the coarse
side evaluated at the images of those points.  Pins:

* the matrix built from unit vectors (the paper's construction, section 3.1)
  equals the independent element/face assembly, and is symmetric positive
  definite;
* constants: A 1 does not depend on beta (no gradient, no jump) and its sum
  is the volume;
* exact reproduction of Q_k polynomials across hanging faces: on an
  all-Neumann box of box cells, A I(p) equals int (a p - b lap p) phi_i +
  int_bdry b dn p phi_i built here from 1-D integrals (every integrand is
  exact with (k+1) Gauss points, also on the quarter faces, where the coarse
  side's test functions are polynomials of degree k in the fine face's
  coordinates);
* manufactured solutions converge at order k+1 on refined periodic meshes
  (affine and curved);
* plausible mistakes planted in the oracle (the quarter's two halves
  exchanged, the coarse points not halved, minus and plus swapped) fail the
  reproduction pin.
"""
import ctypes
import math
import subprocess

import numpy as np
import pytest

import oracle
import oracle.core as oc
import synth_inputs as si


def _np_rules(n):
    xq, wq = np.polynomial.legendre.leggauss(n)
    xq, wq = 0.5 * (xq + 1), 0.5 * wq
    r = np.polynomial.legendre.Legendre.basis(n - 1).deriv().roots() if n > 2 else np.array([])
    xl = np.concatenate([[0.0], 0.5 * (np.sort(r) + 1), [1.0]])
    return xq, wq, xl


def _np_lagrange(xl, t):
    n = xl.size
    C = np.linalg.inv(np.vander(xl, n, increasing=True))
    pw = np.array([t ** m for m in range(n)])
    dpw = np.array([m * t ** (m - 1) if m > 0 else 0.0 for m in range(n)])
    return pw @ C, dpw @ C


def _tiny_refined():
    return [
        ("2x2x2-periodic", si.refined_mesh(2, 2, 2, ((0, 1), (0, 1), (0, 1)))),
        ("3x2x2-neumann", si.refined_mesh(3, 2, 2, ((1, 2), (0, 1), (0, 1)), periodic=(False,) * 3)),
        ("2x1x2-sheared", si.refined_mesh(2, 1, 2, ((0, 1), (0, 1), (1, 2)), periodic=(True, True, False),
                                          mapping=si.random_affine_mapping(3))),
        ("terrain", si.refined_terrain_mesh(4, 1, 2, g=2, region=((1, 2), (0, 1), (0, 1)))),
    ]


def test_refined_meshes_are_valid():
    for name, m in _tiny_refined():
        p = oracle.Problem(m, 1)
        assert p.mesh_check() == 0, name
        assert m.hang.shape[0] > 0 and m.hang.shape[0] % 4 == 0, name
        # every marked face is listed once from the fine side and four times
        # (distinct quarters) from the coarse side
        for c in range(m.n_cells):
            for f in range(6):
                if m.nbr[c, f] != -2:
                    continue
                fine = (m.hang[:, 2] == c) & (m.hang[:, 1] == (f ^ 1))
                coarse = (m.hang[:, 0] == c) & (m.hang[:, 1] == f)
                assert fine.sum() + coarse.sum() in (1, 4), (name, c, f)
                if coarse.sum():
                    assert sorted(m.hang[coarse, 3]) == [0, 1, 2, 3]
        assert (p.hang_sigma() > 0).all()


@pytest.mark.parametrize("k", [1, 2, 3])
def test_hanging_unit_vector_matrix_equals_assembly(k):
    for name, m in _tiny_refined():
        if k == 3 and m.n_cells > 12:
            continue
        p = oracle.Problem(m, k)
        fa, fb = si.terrain_coefficients() if name == "terrain" else si.random_smooth_coefficients(k)
        p.set_coefficient_functions(fa, fb)
        A1 = p.matrix_by_unit_vectors()
        A2 = p.assemble_dense()
        scale = np.abs(A2).max()
        assert np.abs(A1 - A2).max() <= 1e-13 * scale, name
        assert np.abs(A2 - A2.T).max() <= 1e-14 * scale, name
        assert np.linalg.eigvalsh(0.5 * (A2 + A2.T)).min() > 0, name
        # the face terms alone also match (the hanging terms are face terms)
        F1 = p.matrix_by_unit_vectors(oracle.OR_FACE)
        F2 = p.assemble_dense(oracle.OR_FACE)
        assert np.abs(F1 - F2).max() <= 1e-13 * scale, name
        assert np.abs(F2).max() > 1e-3 * scale


def test_hanging_constants_and_volume():
    for name, m in _tiny_refined():
        p = oracle.Problem(m, 2)
        fa, fb = si.random_smooth_coefficients(2)
        p.set_coefficient_functions(fa, fb)
        y1 = p.apply(np.ones(p.n_dofs))
        p.set_coefficient_functions(fa, lambda x, y, z: 5.0 * fb(x, y, z) + 1.0)
        y2 = p.apply(np.ones(p.n_dofs))
        assert np.abs(y1 - y2).max() <= 1e-13 * np.abs(y1).max(), name
    m = si.refined_mesh(3, 2, 2, ((1, 2), (0, 1), (0, 2)), periodic=(False,) * 3)
    p = oracle.Problem(m, 3)
    p.set_coefficient_functions(*si.const_coefficients(1.0, 0.3))
    assert abs(p.apply(np.ones(p.n_dofs)).sum() - 1.0) < 1e-13


def _box_cells(m):
    """origin and size of every (box) cell from its corner nodes (g = 1)."""
    X = m.nodes
    return X[:, 0, :], X[:, -1, :] - X[:, 0, :]


def _reproduction_error(k, m, seed=1, alpha=0.7, beta=0.3):
    rng = np.random.default_rng(seed)
    n = k + 1
    p = oracle.Problem(m, k)
    p.set_coefficient_functions(*si.const_coefficients(alpha, beta))
    q = [np.polynomial.Polynomial(rng.normal(size=k + 1)) for _ in range(3)]
    xyz = p.dof_coords()
    u = q[0](xyz[0]) * q[1](xyz[1]) * q[2](xyz[2])
    Au = p.apply(u)
    xq, wq, xl = _np_rules(n)
    org, siz = _box_cells(m)
    b = np.zeros(p.n_dofs)
    for cell in range(m.n_cells):
        I = []
        for d in range(3):
            i0 = np.zeros(n); i2 = np.zeros(n)
            for x, w in zip(xq, wq):
                v, _ = _np_lagrange(xl, x)
                X = org[cell, d] + siz[cell, d] * x
                i0 += w * siz[cell, d] * q[d](X) * v
                i2 += w * siz[cell, d] * q[d].deriv(2)(X) * v
            I.append((i0, i2))
        loc = np.zeros((n, n, n))
        for l in range(n):
            for j in range(n):
                for i in range(n):
                    val = alpha * I[0][0][i] * I[1][0][j] * I[2][0][l]
                    lap = (I[0][1][i] * I[1][0][j] * I[2][0][l] + I[0][0][i] * I[1][1][j] * I[2][0][l]
                           + I[0][0][i] * I[1][0][j] * I[2][1][l])
                    loc[l, j, i] = val - beta * lap
        for d in range(3):
            for end in (0, 1):
                if m.nbr[cell, 2 * d + end] != -1:
                    continue
                X = org[cell, d] + end * siz[cell, d]
                dn = (1.0 if end else -1.0) * q[d].deriv(1)(X)
                li = 0 if end == 0 else n - 1
                others = [e for e in range(3) if e != d]
                for a in range(n):
                    for c2 in range(n):
                        idx = [0, 0, 0]
                        idx[d] = li; idx[others[0]] = a; idx[others[1]] = c2
                        loc[idx[2], idx[1], idx[0]] += beta * dn * I[others[0]][0][a] * I[others[1]][0][c2]
        b[cell * n ** 3:(cell + 1) * n ** 3] = loc.ravel()
    return np.abs(Au - b).max() / np.abs(b).max()


def _neumann_refined():
    # refined block touching interior faces in all three directions
    return si.refined_mesh(3, 3, 2, ((1, 2), (0, 2), (0, 1)), lo=(0, 0, 0), hi=(1.5, 1.2, 0.8),
                           periodic=(False,) * 3)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_hanging_polynomial_reproduction(k):
    assert _reproduction_error(k, _neumann_refined()) <= 1e-12


def _quad_err(p, u, fexact):
    xyz, w = p.quad_data()
    uq = np.zeros(p.n_dofs)
    oc.lib().or_eval_quad(p._s(), oc._dp(np.ascontiguousarray(u)), oc._dp(uq))
    return math.sqrt(np.sum(w * (uq - fexact(*xyz)) ** 2))


@pytest.mark.slow
@pytest.mark.parametrize("k,sizes,curved", [(2, (2, 4, 8), False), (3, (2, 4), False), (2, (2, 4, 8), True)])
def test_hanging_manufactured_solution_rates(k, sizes, curved):
    tp = 2 * math.pi
    alpha, beta = 1.0, 0.05

    def uex(x, y, z):
        return np.sin(tp * x) * np.cos(tp * y) * np.sin(tp * z + 0.3)

    def f(x, y, z):
        return (alpha + beta * 3 * tp * tp) * uex(x, y, z)
    errs = []
    for nc in sizes:
        region = ((nc // 4, max(nc // 4 + 1, 3 * nc // 4)), (0, nc), (0, max(1, nc // 2)))
        m = si.refined_mesh(nc, nc, nc, region, g=k if curved else 1,
                            mapping=si.wavy_mapping(0.03) if curved else None)
        p = oracle.Problem(m, k)
        p.set_coefficient_functions(*si.const_coefficients(alpha, beta))
        b = p.load_vector(f)
        x, info = oracle.solvers.cg(p.apply, b, precond=p.bj_apply, rtol=1e-12, max_iter=3000)
        assert info.converged
        errs.append(_quad_err(p, x, uex))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print(f"[mms hanging] k={k} curved={curved} errors {errs} rates {rates}")
    assert rates[-1] > k + 1 - 0.35, (errs, rates)


def test_hanging_block_jacobi_is_spd_and_uses_the_quarter_penalties():
    m = si.refined_terrain_mesh(4, 1, 2, g=2, region=((1, 2), (0, 1), (0, 1)))
    p = oracle.Problem(m, 2)
    p.set_coefficient_functions(*si.terrain_coefficients())
    hs = p.hang_sigma()
    for c in range(m.n_cells):
        Ab = p.bj_sep_block(c)
        assert np.abs(Ab - Ab.T).max() <= 1e-14 * np.abs(Ab).max()
        assert np.linalg.eigvalsh(Ab).min() > 0
        _, _, _, sig = p.bj_cell_data(c)
        for f in range(6):
            if m.nbr[c, f] == -2:
                fine = np.nonzero((m.hang[:, 2] == c) & (m.hang[:, 1] == (f ^ 1)))[0]
                if fine.size:
                    assert abs(sig[f // 2, f % 2] - hs[fine[0]]) <= 1e-13 * hs[fine[0]]
                else:
                    quarters = np.nonzero((m.hang[:, 0] == c) & (m.hang[:, 1] == f))[0]
                    assert hs[quarters].min() * (1 - 1e-13) <= sig[f // 2, f % 2] <= hs[quarters].max() * (1 + 1e-13)


# ---------------------------------------------------------------------------
# planted mistakes
# ---------------------------------------------------------------------------

PLANTS = {
    "halves_exchanged": [("xiC[t1] = 0.5 * ((s & 1) + r->xq[a]);", "xiC[t1] = 0.5 * ((s >> 1) + r->xq[a]);"),
                         ("xiC[t2] = 0.5 * ((s >> 1) + r->xq[b]);", "xiC[t2] = 0.5 * ((s & 1) + r->xq[b]);")],
    "not_halved": [("xiC[t1] = 0.5 * ((s & 1) + r->xq[a]);", "xiC[t1] = r->xq[a];"),
                   ("xiC[t2] = 0.5 * ((s >> 1) + r->xq[b]);", "xiC[t2] = r->xq[b];")],
    "minus_plus_swapped": [("const int minus = (h[1] & 1) ? 0 : 1;   /* the coarse cell is minus on its own +d face */",
                            "const int minus = (h[1] & 1) ? 1 : 0;")],
}


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_hanging_pins_catch_planted_mistakes(plant, tmp_path, monkeypatch):
    src = open(oc.SRC).read()
    for old, new in PLANTS[plant]:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    c = tmp_path / f"{plant}.c"
    so = tmp_path / f"{plant}.so"
    c.write_text(src)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                           "-ffp-contract=off", "-I" + oc.HERE, str(c), "-o", str(so), "-lm"])
    monkeypatch.setattr(oc, "_lib", oc.bind(ctypes.CDLL(str(so))))
    assert _reproduction_error(2, _neumann_refined()) > 1e-4
