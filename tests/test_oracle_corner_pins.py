"""Pins of the oracle's choices where neighbouring cells differ and where the
separable block leaves the affine, constant-coefficient case.

* Face penalty: sigma_F = P (k+1)^2 max(|F|/|K-|, |F|/|K+|).  On a graded
  Cartesian mesh (box cells of unequal widths) |F|/|K| = 1/h_d, so
  sigma_F = P (k+1)^2 / min(h-, h+) in closed form, and the assembled matrix
  equals a Kronecker form built here from 1-D physical SIP matrices with one
  penalty per face (numpy's own Gauss rule, per-cell widths).
* Separable block data: l_d is the mean over the cell's Gauss points of the
  column norm |J e_d|, and alpha_bar, beta_bar are volume-weighted means.  On
  a wedge cell (x' = x (1 + c z): detJ varies, J is not symmetric) both have
  closed forms for linear coefficient fields; on a sheared affine cell l_d is
  h_d |A e_d| for the known matrix A.
* Each pin is shown to fail on a copy of the oracle with a plausible mistake
  planted in its source (min instead of max, the own side only, row instead
  of column norms, unweighted means), compiled here on the CPU.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import oracle.core as oc
import synth_inputs as si

P = 2.0


# ---------------------------------------------------------------------------
# planted variants of the oracle
# ---------------------------------------------------------------------------

def _variant(tmp_path, name, subs):
    src = open(oc.SRC).read()
    for old, new in subs:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    c = tmp_path / f"{name}.c"
    so = tmp_path / f"{name}.so"
    c.write_text(src)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-D_GNU_SOURCE", "-ffp-contract=off", "-I" + oc.HERE, str(c), "-o", str(so),
                           "-lm"])
    return oc.bind(ctypes.CDLL(str(so)))


SIGMA_MAX = "double s = area / vm > area / vp ? area / vm : area / vp;"
PLANTS = {
    "sigma_min": [(SIGMA_MAX, "double s = area / vm < area / vp ? area / vm : area / vp;")],
    "sigma_own": [(SIGMA_MAX, "double s = area / vm;")],
    "ell_rows": [("ell[d] += sqrt(J[0][d] * J[0][d] + J[1][d] * J[1][d] + J[2][d] * J[2][d]);",
                  "ell[d] += sqrt(J[d][0] * J[d][0] + J[d][1] * J[d][1] + J[d][2] * J[d][2]);")],
    "mean_unweighted": [("sa += w * field_at(phi, p->alpha + c * nd, nd);",
                         "sa += field_at(phi, p->alpha + c * nd, nd) / nd;"),
                        ("sb += w * field_at(phi, p->beta + c * nd, nd);",
                         "sb += field_at(phi, p->beta + c * nd, nd) / nd;"),
                        ("*abar = sa / vol;", "*abar = sa;"),
                        ("*bbar = sb / vol;", "*bbar = sb;")],
}


# ---------------------------------------------------------------------------
# graded Cartesian mesh and its Kronecker closed form
# ---------------------------------------------------------------------------

AMP = (0.55, 0.4, 0.3)


def _grade(t, a):
    # monotone on [0, 1] (derivative 1 + a cos(2 pi t) > 0), end points fixed
    return t + a * np.sin(2 * np.pi * t) / (2 * np.pi)


def _graded_mesh(dims, periodic):
    def mapping(x, y, z):
        return _grade(x, AMP[0]), _grade(y, AMP[1]), _grade(z, AMP[2])
    return si.box_mesh(*dims, periodic=periodic, g=1, mapping=mapping)


def _widths(n, a):
    t = _grade(np.arange(n + 1) / n, a)
    return np.diff(t)


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


def _sip_1d_phys(h, k, periodic):
    """Physical 1-D mass and SIP matrices on cells of widths h, with the face
    penalty P (k+1)^2 / min(h-, h+) of every interior face."""
    n = k + 1
    xq, wq, xl = _np_rules(n)
    Mh = np.zeros((n, n)); L0 = np.zeros((n, n))
    for x, w in zip(xq, wq):
        v, d = _np_lagrange(xl, x)
        Mh += w * np.outer(v, v); L0 += w * np.outer(d, d)
    v0, d0 = _np_lagrange(xl, 0.0)
    v1, d1 = _np_lagrange(xl, 1.0)
    nc = h.size
    M = np.zeros((nc * n, nc * n)); L = np.zeros((nc * n, nc * n))
    for c in range(nc):
        s = slice(c * n, (c + 1) * n)
        M[s, s] = h[c] * Mh
        L[s, s] += L0 / h[c]
    for c in range(nc):
        cp = c + 1
        if cp == nc:
            if not periodic:
                continue
            cp = 0
        sig = P * n * n / min(h[c], h[cp])
        side = {0: (c, v1, d1 / h[c], 1.0), 1: (cp, v0, d0 / h[cp], -1.0)}
        for st in (0, 1):
            ct, vt, dt, zt = side[st]
            for su in (0, 1):
                cu, vu, du, zu = side[su]
                blk = (-0.5 * np.outer(zt * vt, du) - 0.5 * np.outer(dt, zu * vu)
                       + sig * np.outer(zt * vt, zu * vu))
                L[ct * n:(ct + 1) * n, cu * n:(cu + 1) * n] += blk
    return M, L


def _sigma_closed_form(dims, periodic, k):
    n = k + 1
    hs = [_widths(dims[d], AMP[d]) for d in range(3)]
    nx, ny, nz = dims
    out = np.full((nx * ny * nz, 3), -1.0)
    for cz in range(nz):
        for cy in range(ny):
            for cx in range(nx):
                c = cx + nx * (cy + ny * cz)
                for d, i in enumerate((cx, cy, cz)):
                    j = i + 1
                    if j == dims[d]:
                        if not periodic[d]:
                            continue
                        j = 0
                    out[c, d] = P * n * n / min(hs[d][i], hs[d][j])
    return out


def _graded_kron_error(k, dims, periodic, alpha=1.3, beta=0.02):
    m = _graded_mesh(dims, periodic)
    p = oracle.Problem(m, k, P=P)
    p.set_coefficient_functions(*si.const_coefficients(alpha, beta))
    n = k + 1
    Ms, Ls = [], []
    for d in range(3):
        Md, Ld = _sip_1d_phys(_widths(dims[d], AMP[d]), k, periodic[d])
        Ms.append(Md); Ls.append(Ld)
    A_k = alpha * np.kron(Ms[2], np.kron(Ms[1], Ms[0])) + beta * (
        np.kron(Ms[2], np.kron(Ms[1], Ls[0])) + np.kron(Ms[2], np.kron(Ls[1], Ms[0]))
        + np.kron(Ls[2], np.kron(Ms[1], Ms[0])))
    nx, ny, nz = dims
    N1 = (nx * n, ny * n)
    perm = np.empty(p.n_dofs, dtype=np.int64)
    for cz in range(nz):
        for cy in range(ny):
            for cx in range(nx):
                cell = cx + nx * (cy + ny * cz)
                for l in range(n):
                    for j in range(n):
                        for i in range(n):
                            I = (cx * n + i) + N1[0] * ((cy * n + j) + N1[1] * (cz * n + l))
                            perm[cell * n ** 3 + i + n * (j + n * l)] = I
    A_ref = A_k[np.ix_(perm, perm)]
    A = p.assemble_dense()
    return np.abs(A - A_ref).max() / np.abs(A_ref).max()


def _sigma_error(k, dims, periodic):
    p = oracle.Problem(_graded_mesh(dims, periodic), k, P=P)
    s = p.face_sigma()
    ref = _sigma_closed_form(dims, periodic, k)
    return np.abs(s - ref).max() / ref.max()


GRADED = [(2, (4, 3, 2), (True, True, False)), (1, (3, 2, 3), (True, False, True)),
          (3, (3, 2, 2), (False, True, True))]


@pytest.mark.parametrize("k,dims,periodic", GRADED)
def test_penalty_on_graded_mesh_is_the_closed_form(k, dims, periodic):
    # the widths really differ across faces
    h = _widths(dims[0], AMP[0])
    assert h.max() / h.min() > 1.5
    assert _sigma_error(k, dims, periodic) <= 1e-13


@pytest.mark.parametrize("k,dims,periodic", GRADED)
def test_graded_mesh_matrix_is_the_kronecker_form(k, dims, periodic):
    assert _graded_kron_error(k, dims, periodic) <= 1e-13


# ---------------------------------------------------------------------------
# separable block data on a wedge cell and a sheared affine cell
# ---------------------------------------------------------------------------

LX, LY, LZ, CW = 1.5, 0.8, 0.6, 0.9
ACOEF = (1.2, 0.3, -0.4, 0.5)       # alpha = a0 + a1 x + a2 y + a3 z
BCOEF = (0.05, -0.01, 0.02, 0.03)


def _linear(cf):
    return lambda x, y, z: cf[0] + cf[1] * x + cf[2] * y + cf[3] * z


def _wedge_problem(k):
    m = si.box_mesh(1, 1, 1, lo=(0, 0, 0), hi=(LX, LY, LZ), periodic=(False,) * 3, g=1,
                    mapping=lambda x, y, z: (x * (1 + CW * z), y, z))
    p = oracle.Problem(m, k)
    p.set_coefficient_functions(_linear(ACOEF), _linear(BCOEF))
    return p


def _wedge_closed_forms(k):
    """l_d and the volume-weighted means of linear fields on the wedge
    x' = LX xi0 (1 + b xi2), y' = LY xi1, z' = LZ xi2 with b = CW LZ."""
    n = k + 1
    xq, _, _ = _np_rules(n)
    b = CW * LZ
    ell0 = LX * (1 + b * xq.mean())
    ell1 = LY
    xi0, xi2 = np.meshgrid(xq, xq, indexing="ij")
    ell2 = np.mean(np.sqrt((CW * LX * LZ * xi0) ** 2 + LZ ** 2))
    vol = 1 + b / 2                                  # int (1 + b xi2), times LX LY LZ

    def wmean(cf):
        a0, a1, a2, a3 = cf
        s = (a0 * (1 + b / 2) + a1 * LX * 0.5 * (1 + b + b * b / 3)
             + a2 * LY * 0.5 * (1 + b / 2) + a3 * LZ * (0.5 + b / 3))
        return s / vol
    return np.array([ell0, ell1, ell2]), wmean(ACOEF), wmean(BCOEF)


def _wedge_errors(k):
    p = _wedge_problem(k)
    ell, ab, bb, sig = p.bj_cell_data(0)
    ell_r, ab_r, bb_r = _wedge_closed_forms(k)
    assert (sig < 0).all()                           # a single Neumann cell
    return (np.abs(ell - ell_r).max() / ell_r.max(), abs(ab - ab_r) / abs(ab_r),
            abs(bb - bb_r) / abs(bb_r))


def _sheared_error(k):
    f = si.random_affine_mapping(4, amp=0.3)
    A = np.array([f(*e) for e in np.eye(3)]).T - np.array(f(0.0, 0.0, 0.0))[:, None]
    hi = (0.7, 0.5, 0.4)
    m = si.box_mesh(1, 1, 1, lo=(0, 0, 0), hi=hi, periodic=(False,) * 3, g=1, mapping=f)
    p = oracle.Problem(m, k)
    p.set_coefficient_functions(_linear(ACOEF), _linear(BCOEF))
    ell, ab, bb, _ = p.bj_cell_data(0)
    ell_r = np.array([hi[d] * np.linalg.norm(A[:, d]) for d in range(3)])
    # affine cell: the volume-weighted mean of a linear field is its value at
    # the centroid, the image of the reference centre
    cen = f(*(0.5 * np.array(hi)))
    ab_r = _linear(ACOEF)(*cen)
    return max(np.abs(ell - ell_r).max() / ell_r.max(), abs(ab - ab_r) / abs(ab_r))


@pytest.mark.parametrize("k", [1, 2, 4])
def test_bj_cell_data_on_a_wedge_cell(k):
    e_ell, e_a, e_b = _wedge_errors(k)
    assert e_ell <= 1e-14 and e_a <= 1e-13 and e_b <= 1e-13


@pytest.mark.parametrize("k", [1, 3])
def test_bj_cell_data_on_a_sheared_affine_cell(k):
    assert _sheared_error(k) <= 1e-13


def test_bj_block_on_the_wedge_uses_those_scalars():
    """The separable block is the Kronecker form of the pinned scalars:
    abar lx ly lz M(x)M(x)M + bbar [(ly lz/lx) M(x)M(x)L + ...] with the 1-D
    reference matrices built here (all ends Neumann: L is the plain stiffness)."""
    k = 2
    n = k + 1
    p = _wedge_problem(k)
    ell, ab, bb = _wedge_closed_forms(k)
    xq, wq, xl = _np_rules(n)
    Mh = np.zeros((n, n)); L0 = np.zeros((n, n))
    for x, w in zip(xq, wq):
        v, d = _np_lagrange(xl, x)
        Mh += w * np.outer(v, v); L0 += w * np.outer(d, d)
    lx, ly, lz = ell
    K = lambda a, b_, c: np.kron(c, np.kron(b_, a))     # x fastest
    ref = (ab * lx * ly * lz * K(Mh, Mh, Mh) + bb * (ly * lz / lx * K(L0, Mh, Mh)
           + lx * lz / ly * K(Mh, L0, Mh) + lx * ly / lz * K(Mh, Mh, L0)))
    Ab = p.bj_sep_block(0)
    assert np.abs(Ab - ref).max() <= 1e-13 * np.abs(ref).max()


# ---------------------------------------------------------------------------
# the pins catch plausible mistakes planted in the oracle
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("plant", ["sigma_min", "sigma_own"])
def test_penalty_pins_catch_planted_mistakes(plant, tmp_path, monkeypatch):
    monkeypatch.setattr(oc, "_lib", _variant(tmp_path, plant, PLANTS[plant]))
    k, dims, periodic = GRADED[0]
    assert _sigma_error(k, dims, periodic) > 1e-3
    assert _graded_kron_error(k, dims, periodic) > 1e-3


@pytest.mark.parametrize("plant", ["ell_rows", "mean_unweighted"])
def test_block_data_pins_catch_planted_mistakes(plant, tmp_path, monkeypatch):
    monkeypatch.setattr(oc, "_lib", _variant(tmp_path, plant, PLANTS[plant]))
    e_ell, e_a, e_b = _wedge_errors(2)
    if plant == "ell_rows":
        assert e_ell > 1e-3
        assert _sheared_error(2) > 1e-3
    else:
        assert e_a > 1e-3 and e_b > 1e-3
