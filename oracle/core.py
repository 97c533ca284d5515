"""ctypes front-end of the C oracle (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this module.  It compiles ``oracle.c`` with gcc on demand (``build()``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")

OR_CELL = 1
OR_FACE = 2
OR_ALL = 3


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (gcc, OpenMP, FP64)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-D_GNU_SOURCE", "-ffp-contract=off", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd, cwd=HERE)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _Prob(C.Structure):
    _fields_ = [("k", C.c_int), ("g", C.c_int), ("n_cells", C.c_long),
                ("nodes", C.c_void_p), ("nbr", C.c_void_p),
                ("alpha", C.c_void_p), ("beta", C.c_void_p), ("P", C.c_double),
                ("n_hang", C.c_long), ("hang", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = bind(C.CDLL(LIB))
    return _lib


def bind(L):
    """Declare the argument types of the oracle's entry points on a loaded
    copy of the library (the oracle itself, or a variant a test compiled)."""
    dp = C.POINTER(C.c_double)
    pp = C.POINTER(_Prob)
    L.or_gauss_legendre.argtypes = [C.c_int, dp, dp]
    L.or_gauss_lobatto.argtypes = [C.c_int, dp, dp]
    L.or_lagrange.argtypes = [C.c_int, dp, C.c_double, dp, dp]
    L.or_mesh_check.argtypes = [pp]
    L.or_mesh_check.restype = C.c_int
    for name in ("or_dof_coords", "or_cell_volumes", "or_face_sigma", "or_hang_sigma"):
        getattr(L, name).argtypes = [pp, dp]
    L.or_quad_data.argtypes = [pp, dp, dp]
    L.or_load_vector.argtypes = [pp, dp, dp]
    L.or_apply.argtypes = [pp, C.c_int, dp, dp]
    L.or_assemble_dense.argtypes = [pp, C.c_int, dp]
    L.or_cell_diagonal.argtypes = [pp, C.c_int, dp]
    L.or_mass_block.argtypes = [pp, C.c_long, dp]
    L.or_mass_block_apply.argtypes = [pp, dp, dp]
    L.or_mass_block_apply.restype = C.c_int
    L.or_grad_apply.argtypes = [pp, C.c_double, dp, dp]
    L.or_apply_q.argtypes = [pp, C.c_int, C.c_int, dp, dp]
    L.or_apply_q_cells.argtypes = [pp, C.c_int, C.c_int, C.c_void_p, C.c_long, dp, dp]
    L.or_div_apply.argtypes = [pp, C.c_double, dp, dp, dp]
    L.or_grad_apply_cells.argtypes = [pp, C.c_double, C.c_void_p, C.c_long, dp, dp]
    L.or_div_apply_cells.argtypes = [pp, C.c_double, dp, C.c_void_p, C.c_long, dp, dp]
    L.or_apply_cells.argtypes = [pp, C.c_int, C.c_void_p, C.c_long, dp, dp]
    L.or_bj_cell_data.argtypes = [pp, C.c_long, dp, dp, dp, dp]
    L.or_bj_sep_block.argtypes = [pp, C.c_long, dp]
    L.or_bj_sep_apply.argtypes = [pp, dp, dp]
    L.or_bj_sep_apply.restype = C.c_int
    return L


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ---------------------------------------------------------------------------
# 1-D rules
# ---------------------------------------------------------------------------

def gauss_legendre(n: int):
    x = np.zeros(n); w = np.zeros(n)
    lib().or_gauss_legendre(n, _dp(x), _dp(w))
    return x, w


def gauss_lobatto(n: int):
    x = np.zeros(n); w = np.zeros(n)
    lib().or_gauss_lobatto(n, _dp(x), _dp(w))
    return x, w


def lagrange(nodes: np.ndarray, t: float):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    n = nodes.size
    v = np.zeros(n); d = np.zeros(n)
    lib().or_lagrange(n, _dp(nodes), float(t), _dp(v), _dp(d))
    return v, d


# ---------------------------------------------------------------------------
# problem
# ---------------------------------------------------------------------------

class Problem:
    """A mesh, a degree and (optionally) coefficient fields, as the oracle sees
    them.  Arrays are kept alive here; ``alpha``/``beta`` are DG nodal fields
    ``[n_cells*(k+1)^3]``."""

    def __init__(self, mesh, k: int, alpha=None, beta=None, P: float = 2.0):
        self.mesh = mesh
        self.k = int(k)
        self.g = int(mesh.g)
        self.n = self.k + 1
        self.nd = self.n ** 3
        self.n_cells = mesh.n_cells
        self.n_dofs = self.n_cells * self.nd
        self.nodes = np.ascontiguousarray(mesh.nodes, dtype=np.float64)
        self.nbr = np.ascontiguousarray(mesh.nbr, dtype=np.int64)
        hang = getattr(mesh, "hang", None)
        self.hang = np.ascontiguousarray(np.zeros((0, 4)) if hang is None else hang,
                                         dtype=np.int64).reshape(-1, 4)
        self.P = float(P)
        self.alpha = None
        self.beta = None
        if alpha is not None:
            self.set_coefficients(alpha, beta)

    def set_coefficients(self, alpha, beta):
        self.alpha = np.ascontiguousarray(alpha, dtype=np.float64)
        self.beta = np.ascontiguousarray(beta, dtype=np.float64)
        assert self.alpha.shape == (self.n_dofs,) and self.beta.shape == (self.n_dofs,)

    def set_coefficient_functions(self, fa, fb):
        x, y, z = self.dof_coords()
        self.set_coefficients(fa(x, y, z), fb(x, y, z))

    def _s(self):
        zero = None
        s = _Prob(self.k, self.g, self.n_cells,
                  self.nodes.ctypes.data, self.nbr.ctypes.data,
                  self.alpha.ctypes.data if self.alpha is not None else zero,
                  self.beta.ctypes.data if self.beta is not None else zero,
                  self.P, self.hang.shape[0], self.hang.ctypes.data)
        return C.byref(s)

    # geometry ------------------------------------------------------------
    def mesh_check(self) -> int:
        return lib().or_mesh_check(self._s())

    def dof_coords(self):
        xyz = np.zeros(3 * self.n_dofs)
        lib().or_dof_coords(self._s(), _dp(xyz))
        return xyz.reshape(3, self.n_dofs)

    def quad_data(self):
        xyz = np.zeros(3 * self.n_dofs)
        w = np.zeros(self.n_dofs)
        lib().or_quad_data(self._s(), _dp(xyz), _dp(w))
        return xyz.reshape(3, self.n_dofs), w

    def load_vector(self, f):
        """b_i = int f phi_i by the cell GL rule; f is a function of (x,y,z)."""
        xyz, _ = self.quad_data()
        fq = np.ascontiguousarray(f(xyz[0], xyz[1], xyz[2]), dtype=np.float64)
        b = np.zeros(self.n_dofs)
        lib().or_load_vector(self._s(), _dp(fq), _dp(b))
        return b

    def hang_sigma(self):
        """Penalty of every non-conforming quarter face (hanging record)."""
        s = np.zeros(self.hang.shape[0])
        if s.size:
            lib().or_hang_sigma(self._s(), _dp(s))
        return s

    def cell_volumes(self):
        v = np.zeros(self.n_cells)
        lib().or_cell_volumes(self._s(), _dp(v))
        return v

    def face_sigma(self):
        s = np.zeros(3 * self.n_cells)
        lib().or_face_sigma(self._s(), _dp(s))
        return s.reshape(self.n_cells, 3)

    # operator ------------------------------------------------------------
    def apply(self, x, flags: int = OR_ALL):
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n_dofs)
        lib().or_apply(self._s(), int(flags), _dp(x), _dp(y))
        return y

    def apply_q(self, x, nq: int, flags: int = OR_ALL):
        """A x with an nq-point Gauss rule per direction (nq = 2k+1:
        consistent integration)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros(self.n_dofs)
        lib().or_apply_q(self._s(), int(nq), int(flags), _dp(x), _dp(y))
        return y

    def apply_q_cells(self, x, cells, nq: int, flags: int = OR_ALL):
        x = np.ascontiguousarray(x, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros(cells.size * self.nd)
        lib().or_apply_q_cells(self._s(), int(nq), int(flags), cells.ctypes.data, cells.size,
                               _dp(x), _dp(out))
        return out.reshape(cells.size, self.nd)

    def apply_cells(self, x, cells, flags: int = OR_ALL):
        """(A x) restricted to the listed cells: [len(cells), nd]."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros(cells.size * self.nd)
        lib().or_apply_cells(self._s(), int(flags), cells.ctypes.data, cells.size, _dp(x), _dp(out))
        return out.reshape(cells.size, self.nd)

    def assemble_dense(self, flags: int = OR_ALL):
        A = np.zeros((self.n_dofs, self.n_dofs))
        lib().or_assemble_dense(self._s(), int(flags), _dp(A))
        return A

    def matrix_by_unit_vectors(self, flags: int = OR_ALL):
        """Columns A e_j, one operator application per unit vector."""
        A = np.zeros((self.n_dofs, self.n_dofs))
        e = np.zeros(self.n_dofs)
        for j in range(self.n_dofs):
            e[j] = 1.0
            A[:, j] = self.apply(e, flags)
            e[j] = 0.0
        return A

    # the paper's diagonal preconditioners ---------------------------------
    def cell_diagonal(self, stiff: bool = True):
        """Diagonal of the volume part of the form (mass plus stiffness, or the
        mass alone): the matrices whose inverses are the paper's Helmholtz and
        internal-energy preconditioners (section 3.1)."""
        d = np.zeros(self.n_dofs)
        lib().or_cell_diagonal(self._s(), int(bool(stiff)), _dp(d))
        return d

    def mass_block(self, c: int):
        """The alpha-weighted mass matrix of cell c (direct quadrature)."""
        M = np.zeros(self.nd * self.nd)
        lib().or_mass_block(self._s(), int(c), _dp(M))
        return M.reshape(self.nd, self.nd)

    def mass_block_apply(self, r):
        """z = M^{-1} r with M the block-diagonal alpha-weighted mass matrix."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.n_dofs)
        if lib().or_mass_block_apply(self._s(), _dp(r), _dp(z)):
            raise FloatingPointError("mass block not positive definite")
        return z

    # velocity-pressure coupling -------------------------------------------
    def grad_apply(self, p, tau: float = 1.0):
        """B p (pressure gradient with central flux, own trace on boundary
        faces), scaled by tau: [3, n_dofs]."""
        p = np.ascontiguousarray(p, dtype=np.float64)
        u3 = np.zeros(3 * self.n_dofs)
        lib().or_grad_apply(self._s(), float(tau), _dp(p), _dp(u3))
        return u3.reshape(3, self.n_dofs)

    def div_apply(self, u3, hr, tau: float = 1.0):
        """C u (divergence of hr u with central flux, no boundary flux),
        scaled by tau; u3 is [3, n_dofs], hr a nodal field."""
        u3 = np.ascontiguousarray(u3, dtype=np.float64).reshape(-1)
        hr = np.ascontiguousarray(hr, dtype=np.float64)
        q = np.zeros(self.n_dofs)
        lib().or_div_apply(self._s(), float(tau), _dp(hr), _dp(u3), _dp(q))
        return q

    def grad_cells(self, p, cells, tau: float = 1.0):
        """B p on the listed cells only: [len(cells), 3, nd]."""
        p = np.ascontiguousarray(p, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros(cells.size * 3 * self.nd)
        lib().or_grad_apply_cells(self._s(), float(tau), cells.ctypes.data, cells.size, _dp(p), _dp(out))
        return out.reshape(cells.size, 3, self.nd)

    def div_cells(self, u3, hr, cells, tau: float = 1.0):
        """C u on the listed cells only (u3 [3, n_dofs] needs valid values on
        those cells and their face neighbours): [len(cells), nd]."""
        u3 = np.ascontiguousarray(u3, dtype=np.float64).reshape(-1)
        hr = np.ascontiguousarray(hr, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.zeros(cells.size * self.nd)
        lib().or_div_apply_cells(self._s(), float(tau), _dp(hr), cells.ctypes.data, cells.size,
                                 _dp(u3), _dp(out))
        return out.reshape(cells.size, self.nd)

    # block Jacobi ----------------------------------------------------------
    def bj_cell_data(self, c: int):
        ell = np.zeros(3); ab = np.zeros(1); bb = np.zeros(1); sig = np.zeros(6)
        lib().or_bj_cell_data(self._s(), int(c), _dp(ell), _dp(ab), _dp(bb), _dp(sig))
        return ell, float(ab[0]), float(bb[0]), sig.reshape(3, 2)

    def bj_sep_block(self, c: int):
        A = np.zeros(self.nd * self.nd)
        lib().or_bj_sep_block(self._s(), int(c), _dp(A))
        return A.reshape(self.nd, self.nd)

    def bj_apply(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.zeros(self.n_dofs)
        bad = lib().or_bj_sep_apply(self._s(), _dp(r), _dp(z))
        if bad:
            raise FloatingPointError("separable block not positive definite")
        return z


class PressureSystem:
    """The pressure system of one IMEX stage (section 2):
        A U + B P = F,   C U + D P = G,
        S P = D P - C A^-1 B P = G - C A^-1 F,
    with A the rho-weighted velocity mass (one scalar block per component),
    B the tau-scaled pressure gradient, C the tau-scaled divergence of
    (h rho) u, D the internal-energy mass of an ideal gas, (1/(gamma-1)) M.
    Composed from the oracle's own operators, in the paper's order."""

    def __init__(self, mesh, k: int, rho, h, gamma: float, tau: float):
        self.vel = Problem(mesh, k, alpha=rho, beta=np.zeros_like(rho))
        n = self.vel.n_dofs
        self.pmass = Problem(mesh, k, alpha=np.full(n, 1.0 / (gamma - 1.0)), beta=np.zeros(n))
        self.hr = np.ascontiguousarray(np.asarray(h) * np.asarray(rho), dtype=np.float64)
        self.tau = float(tau)
        self.n_dofs = n

    def a_inv(self, u3):
        return np.stack([self.vel.mass_block_apply(u3[c]) for c in range(3)])

    def grad(self, p):
        return self.vel.grad_apply(p, self.tau)

    def div(self, u3):
        return self.vel.div_apply(u3, self.hr, self.tau)

    def d_apply(self, p):
        return self.pmass.apply(p, OR_CELL)

    def apply(self, p):
        return self.d_apply(p) - self.div(self.a_inv(self.grad(p)))

    def rhs(self, F, G):
        return np.asarray(G) - self.div(self.a_inv(np.asarray(F)))

    def velocity(self, F, p):
        return self.a_inv(np.asarray(F) - self.grad(p))

    def apply_cells(self, p, cells):
        """S p on the listed cells only, from the cells' two-layer stencil:
        B p on the cells and their face neighbours, A^-1 per cell by a dense
        solve of its mass block, C on the cells, D p on the cells."""
        cells = np.asarray(cells, dtype=np.int64)
        nbr = self.vel.nbr
        stencil = np.unique(np.concatenate([cells, nbr[cells].ravel()]))
        stencil = stencil[stencil >= 0]
        nd, n = self.vel.nd, self.n_dofs
        bp = self.vel.grad_cells(p, stencil, self.tau)          # [ms, 3, nd]
        v3 = np.zeros((3, n))
        for s, c in enumerate(stencil):
            Mb = self.vel.mass_block(int(c))
            v3[:, c * nd:(c + 1) * nd] = np.linalg.solve(Mb, bp[s].T).T
        cq = self.vel.div_cells(v3, self.hr, cells, self.tau)   # [m, nd]
        dq = self.pmass.apply_cells(p, cells, OR_CELL)
        return dq - cq
