"""Plain FP64 Krylov solvers of the oracle (test infrastructure only).

The paper solves its symmetric positive-definite systems with preconditioned
conjugate gradients and its non-symmetric pressure system with GMRES plus a
Jacobi-type preconditioner (section 3.1).  These are the textbook forms:

* ``cg``: preconditioned CG, z = M^{-1} r, stopping on ||r||_2 <= rtol ||b||_2
  (Euclidean norm of the coefficient vector), then re-checking b - A x.
* ``fgmres``: right-preconditioned flexible GMRES(m) (Saad 1993), modified
  Gram-Schmidt, Givens rotations, explicit residual at every restart.  An
  optional stall rule switches the preconditioner to a fallback: if the
  residual estimate over the last ``stall_window`` iterations has not fallen
  below ``stall_ratio`` times its earlier value, or a preconditioned vector is
  not finite, the solver restarts from the current x with the fallback.
* ``ir_solve``: an outer FGMRES whose preconditioner is an inner solve.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class SolveInfo:
    iters: int = 0
    restarts: int = 0
    converged: bool = False
    true_rel_res: float = math.nan
    fallback_used: bool = False
    history: List[float] = field(default_factory=list)


def cg(apply: Callable, b: np.ndarray, precond: Optional[Callable] = None,
       rtol: float = 1e-10, max_iter: int = 10000, x0=None):
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply(x)
    nb = np.linalg.norm(b)
    info = SolveInfo()
    if nb == 0.0:
        info.converged = True
        info.true_rel_res = 0.0
        return x, info
    z = precond(r) if precond else r.copy()
    p = z.copy()
    rz = float(r @ z)
    info.history.append(np.linalg.norm(r) / nb)
    for it in range(max_iter):
        if info.history[-1] <= rtol:
            break
        q = apply(p)
        a = rz / float(p @ q)
        x += a * p
        r -= a * q
        info.iters += 1
        info.history.append(np.linalg.norm(r) / nb)
        if info.history[-1] <= rtol:
            break
        z = precond(r) if precond else r.copy()
        rz_new = float(r @ z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    info.true_rel_res = float(np.linalg.norm(b - apply(x)) / nb)
    info.converged = info.true_rel_res <= rtol * 1.0001 or info.history[-1] <= rtol
    return x, info


def fgmres(apply: Callable, b: np.ndarray, precond: Optional[Callable] = None,
           restart: int = 30, rtol: float = 1e-8, max_iter: int = 5000, x0=None,
           fallback: Optional[Callable] = None, stall_window: int = 10,
           stall_ratio: float = 0.99):
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    nb = np.linalg.norm(b)
    info = SolveInfo()
    if nb == 0.0:
        info.converged, info.true_rel_res = True, 0.0
        return x, info
    M = precond if precond is not None else (lambda v: v.copy())
    m = restart
    while info.iters < max_iter:
        r = b - apply(x)
        beta = np.linalg.norm(r)
        rel = beta / nb
        info.history.append(rel)
        if rel <= rtol:
            info.converged = True
            break
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m); sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_used = 0
        switch = False
        for j in range(m):
            z = M(V[j])
            if not np.all(np.isfinite(z)):
                switch = True
                break
            Z[j] = z
            w = apply(z)
            for i in range(j + 1):          # modified Gram-Schmidt
                H[i, j] = float(w @ V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):              # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            if not (den > 0.0 and math.isfinite(den)):
                switch = True               # breakdown: the space stopped growing
                break
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            info.iters += 1
            j_used = j + 1
            est = abs(g[j + 1]) / nb
            info.history.append(est)
            if est <= rtol:
                break
            if (fallback is not None and not info.fallback_used
                    and len(info.history) > stall_window
                    and est > stall_ratio * info.history[-1 - stall_window]):
                switch = True
                break
            if info.iters >= max_iter:
                break
        if j_used > 0:
            y = np.zeros(j_used)
            for i in range(j_used - 1, -1, -1):
                y[i] = (g[i] - H[i, i + 1:j_used] @ y[i + 1:]) / H[i, i]
            x = x + Z[:j_used].T @ y
        info.restarts += 1
        if switch:
            if fallback is None or info.fallback_used:
                break
            info.fallback_used = True
            M = fallback
    info.true_rel_res = float(np.linalg.norm(b - apply(x)) / nb)
    info.converged = info.true_rel_res <= rtol * 1.0001
    return x, info


def ir_solve(apply: Callable, b: np.ndarray, inner: Callable, restart: int = 10,
             rtol: float = 1e-8, max_iter: int = 500):
    """Outer FP64 FGMRES whose (variable) preconditioner is ``inner(r)``."""
    return fgmres(apply, b, precond=inner, restart=restart, rtol=rtol,
                  max_iter=max_iter)


# ---------------------------------------------------------------------------
# Chebyshev polynomial preconditioning with Lanczos eigenvalue estimates
# (section 3.1 names this technique for the symmetric positive-definite
# systems: a polynomial damping the eigenvalue range, the range estimated
# from the Lanczos process)
# ---------------------------------------------------------------------------

def lanczos_bounds(apply: Callable, precond: Callable, b: np.ndarray, iters: int):
    """Extreme eigenvalues of M^{-1} A from `iters` steps of preconditioned CG
    on A x = b: with step lengths a_k and direction ratios g_k the Lanczos
    matrix is tridiagonal with T[k,k] = 1/a_k + g_{k-1}/a_{k-1} and
    T[k,k+1] = sqrt(g_k)/a_k; its eigenvalues are Ritz values of M^{-1} A."""
    r = np.array(b, dtype=np.float64)
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    al, ga = [], []
    for _ in range(iters):
        q = apply(p)
        a = rz / float(p @ q)
        r = r - a * q
        z = precond(r)
        rz_new = float(r @ z)
        g = rz_new / rz
        al.append(a)
        ga.append(g)
        p = z + g * p
        rz = rz_new
    m = len(al)
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / al[k] + (ga[k - 1] / al[k - 1] if k > 0 else 0.0)
        if k + 1 < m:
            T[k, k + 1] = T[k + 1, k] = math.sqrt(ga[k]) / al[k]
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1])


def chebyshev_apply(apply: Callable, precond: Callable, r: np.ndarray, lo: float, hi: float,
                    degree: int):
    """z = p(M^{-1} A) M^{-1} r: `degree` steps of the Chebyshev iteration for
    A z = r from z = 0 with the interval [lo, hi] of M^{-1} A, so that
    r - A z = T_m((theta - A M^{-1}) / delta) / T_m(theta / delta) r with
    theta = (hi + lo)/2, delta = (hi - lo)/2 (the classical three-term
    recurrence for the scaled Chebyshev polynomials)."""
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = precond(r) / theta
    z = d.copy()
    for _ in range(degree - 1):
        rho_new = 1.0 / (2.0 * sigma - rho)
        res = r - apply(z)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * precond(res)
        z = z + d
        rho = rho_new
    return z
