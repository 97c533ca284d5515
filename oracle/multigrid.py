"""Geometric multigrid of the oracle (test infrastructure only: the tests, the
smoke check and the CPU baseline of the benchmark use it; the GPU path never
does).

Section 3.1 solves the symmetric positive-definite systems with conjugate
gradients preconditioned by geometric multigrid, and names the Chebyshev
polynomial with Lanczos eigenvalue estimates as the matrix-free smoothing
technique.  The paper names the method, not its parts; the reading taken
here is the textbook V-cycle for discontinuous Galerkin spaces:

* levels are uniform refinements: every cell of a finer level lies in one
  octant of a parent cell of the next coarser level, with the same axis
  orientation; the operator is re-discretised on every level at the same
  polynomial degree;
* prolongation writes the coarse function in the fine basis: the child's
  nodal values are the parent polynomial at the child's nodes, mapped into
  the parent's reference cube (the coarse space is a subspace of the fine
  one whenever the geometry is nested);
* restriction is the transpose of prolongation;
* smoothing is the Chebyshev polynomial of M^-1 A (M block Jacobi), the same
  polynomial before and after the coarse-grid correction, so that the
  V-cycle is a symmetric positive-definite operator CG can use;
* the coarsest level applies its own Chebyshev polynomial (over the whole
  estimated range, of a higher degree) in place of an exact solve.

Parity pins: prolongation reproduces polynomials on nested affine meshes;
restriction of the fine mass (and, for continuous fields, of the fine
operator) applied to a prolonged field equals the coarse one (Galerkin
identities that hold exactly there); the V-cycle is symmetric and positive
definite; CG with it needs far fewer iterations than with block Jacobi.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional

import numpy as np

from .core import gauss_lobatto, lagrange, Problem
from . import solvers


def octant_embeddings(k: int) -> np.ndarray:
    """E[o][i][j] = l_j((o + x_i) / 2), o = 0, 1: the coarse Lagrange basis
    (degree k, Gauss-Lobatto nodes on [0, 1]) at the fine nodes of the lower
    (o = 0) and upper (o = 1) half of the parent interval."""
    x, _ = gauss_lobatto(k + 1)
    E = np.zeros((2, k + 1, k + 1))
    for o in (0, 1):
        for i in range(k + 1):
            E[o, i], _ = lagrange(x, 0.5 * (o + x[i]))
    return E


def _bits(octant):
    octant = np.asarray(octant)
    return octant & 1, (octant >> 1) & 1, (octant >> 2) & 1


def prolong(k: int, parent, octant, xc: np.ndarray) -> np.ndarray:
    """Fine nodal vector of the coarse DG function xc (parent[f], octant[f]
    per fine cell f, octant = ox + 2 oy + 4 oz)."""
    n = k + 1
    E = octant_embeddings(k)
    parent = np.asarray(parent)
    Xc = xc.reshape(-1, n, n, n)              # [cell][l][j][i]
    out = np.zeros((parent.size, n, n, n))
    ox, oy, oz = _bits(octant)
    for o in range(8):
        sel = np.nonzero((ox + 2 * oy + 4 * oz) == o)[0]
        if sel.size == 0:
            continue
        Ex, Ey, Ez = E[o & 1], E[(o >> 1) & 1], E[(o >> 2) & 1]
        out[sel] = np.einsum("ia,jb,lc,fcba->flji", Ex, Ey, Ez, Xc[parent[sel]])
    return out.reshape(-1)


def restrict(k: int, parent, octant, rf: np.ndarray, n_coarse: int) -> np.ndarray:
    """Transpose of ``prolong``: coarse dual vector of the fine one."""
    n = k + 1
    E = octant_embeddings(k)
    parent = np.asarray(parent)
    Rf = rf.reshape(-1, n, n, n)
    out = np.zeros((n_coarse, n, n, n))
    ox, oy, oz = _bits(octant)
    for o in range(8):
        sel = np.nonzero((ox + 2 * oy + 4 * oz) == o)[0]
        if sel.size == 0:
            continue
        Ex, Ey, Ez = E[o & 1], E[(o >> 1) & 1], E[(o >> 2) & 1]
        np.add.at(out, parent[sel], np.einsum("ia,jb,lc,flji->fcba", Ex, Ey, Ez, Rf[sel]))
    return out.reshape(-1)


@dataclass
class Level:
    """One level: the problem with its coefficients, its Chebyshev polynomial
    (degree and interval of M^-1 A), and the map of its cells to the next
    coarser level (None on the coarsest)."""
    prob: Problem
    degree: int
    lo: float
    hi: float
    parent: Optional[np.ndarray] = None
    octant: Optional[np.ndarray] = None

    def smooth(self, r):
        return solvers.chebyshev_apply(self.prob.apply, self.prob.bj_apply, r, self.lo, self.hi,
                                       self.degree)


def vcycle(levels: List[Level], b: np.ndarray, l: int = 0) -> np.ndarray:
    """x = V b: pre-smoothing from zero, coarse-grid correction with the
    restricted residual, post-smoothing of the updated residual."""
    L = levels[l]
    if l == len(levels) - 1:
        return L.smooth(b)
    x = L.smooth(b)
    r = b - L.prob.apply(x)
    C = levels[l + 1]
    bc = restrict(L.prob.k, L.parent, L.octant, r, C.prob.n_cells)
    x = x + prolong(L.prob.k, L.parent, L.octant, vcycle(levels, bc, l + 1))
    return x + L.smooth(b - L.prob.apply(x))


def mg_cg(levels: List[Level], b, rtol: float = 1e-8, max_iter: int = 1000):
    """CG on the finest level preconditioned by one V-cycle."""
    return solvers.cg(levels[0].prob.apply, b, precond=lambda r: vcycle(levels, r),
                      rtol=rtol, max_iter=max_iter)
