"""helmdg: matrix-free DG Helmholtz pressure operator and Krylov solve on MI355X.

Thin ctypes binding of ``libhelmdg.so`` (built by ``build.py`` for gfx950).
Every numerical step runs in the library's HIP kernels; this module only
marshals arguments: torch tensors supply device memory and the HIP stream.
Loading fails loudly when the library has not been built -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhelmdg.so")

HX_OK, HX_ERR_ARG, HX_ERR_STATE, HX_ERR_DEVICE, HX_ERR_OOM, HX_ERR_MESH, \
    HX_ERR_NOCONV, HX_FALLBACK_USED = range(8)
HX_F64, HX_F32 = 0, 1
(HX_PC_NONE, HX_PC_BLOCK_JACOBI, HX_PC_LEARNED, HX_PC_HELMHOLTZ_DIAG, HX_PC_MASS_DIAG,
 HX_PC_MASS_BLOCK, HX_PC_CHEBYSHEV, HX_PC_MULTIGRID, HX_PC_MULTIGRID_MIXED) = range(9)
HX_EXPORT_CELL_DATA, HX_EXPORT_FACE_DATA, HX_EXPORT_SIGMA, HX_EXPORT_VOLUME, \
    HX_EXPORT_BJ_SCALARS, HX_EXPORT_INV_DIAG = range(6)
HX_PS_GRAD, HX_PS_DIV, HX_PS_VMASS_INV, HX_PS_DMASS, HX_PS_SYSTEM = range(5)
HX_PART_CELL, HX_PART_FACE = 1, 2
HX_TRACE_INPUT, HX_TRACE_H1, HX_TRACE_H2, HX_TRACE_OUT, HX_TRACE_DOUT, HX_TRACE_DH2, \
    HX_TRACE_DH1 = range(7)

STATUS_NAMES = {0: "HX_OK", 1: "HX_ERR_ARG", 2: "HX_ERR_STATE", 3: "HX_ERR_DEVICE",
                4: "HX_ERR_OOM", 5: "HX_ERR_MESH", 6: "HX_ERR_NOCONV",
                7: "HX_FALLBACK_USED"}


class HXError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class SolveParams(C.Structure):
    _fields_ = [("method", C.c_int), ("restart", C.c_int), ("rtol", C.c_double),
                ("max_iter", C.c_int), ("pc", C.c_int), ("mixed", C.c_int),
                ("inner_iters", C.c_int), ("inner_rtol", C.c_double),
                ("x0_mode", C.c_int), ("stall_window", C.c_int),
                ("stall_ratio", C.c_double), ("orth", C.c_int), ("system", C.c_int)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("restarts", C.c_int), ("status", C.c_int),
                ("fallback_used", C.c_int), ("inner_iters", C.c_int),
                ("true_rel_res", C.c_double), ("ms_total", C.c_double),
                ("ms_op", C.c_double), ("ms_pc", C.c_double), ("ms_orth", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_len", C.c_int)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libhelmdg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} not found: build it with paper_2505_00384_amd/build.py "
                          "(there is no fallback path)")
    L = C.CDLL(path)
    vp, i64, dp = C.c_void_p, C.c_int64, C.POINTER(C.c_double)
    sig = {
        "hx_create": ([C.POINTER(vp), C.c_int, vp], C.c_int),
        "hx_destroy": ([vp], C.c_int),
        "hx_last_error": ([vp], C.c_char_p),
        "hx_max_degree": ([], C.c_int),
        "hx_setup_mesh": ([vp, C.c_int, i64, C.c_int, vp, vp], C.c_int),
        "hx_setup_mesh_hanging": ([vp, C.c_int, i64, C.c_int, vp, vp, i64, vp], C.c_int),
        "hx_dof_coordinates": ([vp, vp], C.c_int),
        "hx_num_dofs": ([vp], i64),
        "hx_set_coefficients": ([vp, vp, vp, C.c_double, C.c_int], C.c_int),
        "hx_apply_operator": ([vp, C.c_int, vp, vp], C.c_int),
        "hx_residual": ([vp, vp, vp, vp], C.c_int),
        "hx_apply_operator_part": ([vp, C.c_int, C.c_int, vp, vp], C.c_int),
        "hx_set_cell_compression": ([vp, C.c_int], C.c_int),
        "hx_operator_info": ([vp, C.c_int, vp, vp], C.c_int),
        "hx_apply_preconditioner": ([vp, C.c_int, C.c_int, vp, vp], C.c_int),
        "hx_default_params": ([C.POINTER(SolveParams)], None),
        "hx_solve": ([vp, C.POINTER(SolveParams), vp, vp, C.POINTER(SolveInfo)], C.c_int),
        "hx_dot": ([vp, i64, vp, vp, dp], C.c_int),
        "hx_network_size": ([vp], i64),
        "hx_set_network": ([vp, vp, i64], C.c_int),
        "hx_get_network": ([vp, vp, i64], C.c_int),
        "hx_gather_features": ([vp, vp, vp, vp], C.c_int),
        "hx_network_forward": ([vp, vp, i64, vp], C.c_int),
        "hx_network_forward_noalloc": ([vp, vp, i64, vp], C.c_int),
        "hx_network_trace": ([vp, C.c_int, vp, i64], C.c_int),
        "hx_network_noalloc_max_batch": ([vp], i64),
        "hx_training_pair": ([vp, vp, vp, vp, C.c_float, vp, vp], C.c_int),
        "hx_train_step": ([vp, vp, vp, i64, C.c_float, C.POINTER(C.c_float), vp], C.c_int),
        "hx_debug_export": ([vp, C.c_int, vp, i64], C.c_int),
        "hx_set_pressure_system": ([vp, vp, vp, C.c_double, C.c_double, C.c_double, C.c_int],
                                   C.c_int),
        "hx_apply_pressure_part": ([vp, C.c_int, vp, vp], C.c_int),
        "hx_set_consistent": ([vp, vp, vp, C.c_int], C.c_int),
        "hx_set_chebyshev": ([vp, C.c_int, C.c_double, C.c_double], C.c_int),
        "hx_estimate_eigenvalues": ([vp, vp, C.c_int, dp, dp], C.c_int),
        "hx_set_multigrid": ([vp, vp, vp, vp], C.c_int),
        "hx_mg_transfer": ([vp, C.c_int, vp, vp], C.c_int),
        "hx_apply_consistent": ([vp, vp, vp], C.c_int),
        "hx_pressure_rhs": ([vp, vp, vp, vp], C.c_int),
        "hx_pressure_velocity": ([vp, vp, vp, vp], C.c_int),
        "hx_solve_pressure_fixed_point": ([vp, vp, vp, vp, vp, C.c_double, C.c_double, C.c_double,
                                           C.POINTER(SolveParams), C.c_int, C.c_double,
                                           C.POINTER(C.c_int), C.POINTER(C.c_double),
                                           C.POINTER(SolveInfo)], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def default_params(**kw) -> SolveParams:
    p = SolveParams()
    load().hx_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _ptr(t) -> int:
    return t.data_ptr()


class HelmDG:
    """One library context on one device, bound to torch's current stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.L = load()
        self.device = device
        torch.cuda.set_device(device)
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        st = self.L.hx_create(C.byref(h), device, C.c_void_p(stream.cuda_stream))
        if st != HX_OK:
            raise HXError(st, "hx_create failed")
        self.h = h
        self.n_dofs = -1
        self.k = None

    # -- helpers ----------------------------------------------------------
    def _chk(self, st: int, what: str):
        if st not in (HX_OK, HX_FALLBACK_USED):
            raise HXError(st, f"{what}: {self.L.hx_last_error(self.h).decode()}")
        return st

    def close(self):
        if getattr(self, "h", None):
            # finer levels that link this one lose the link first
            for fine in list(getattr(self, "_mg_finer", [])):
                f = fine()
                if f is not None and getattr(f, "h", None) and getattr(f, "_mg_coarse", None) is self:
                    f.set_multigrid(None)
            self.L.hx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return self.L.hx_last_error(self.h).decode()

    # -- setup --------------------------------------------------------------
    def setup_mesh(self, degree: int, nodes: np.ndarray, nbr: np.ndarray, geo_degree: int,
                   hang: Optional[np.ndarray] = None):
        """Mesh upload; ``hang`` ([n, 4] int: coarse cell, its face, fine
        cell, quarter) describes non-conforming 2:1 faces marked -2 in nbr."""
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        nbr = np.ascontiguousarray(nbr, dtype=np.int64)
        n_cells = nbr.shape[0]
        if hang is not None and len(hang):
            hang = np.ascontiguousarray(hang, dtype=np.int64).reshape(-1, 4)
            st = self.L.hx_setup_mesh_hanging(self.h, int(degree), n_cells, int(geo_degree),
                                              nodes.ctypes.data, nbr.ctypes.data, hang.shape[0],
                                              hang.ctypes.data)
        else:
            st = self.L.hx_setup_mesh(self.h, int(degree), n_cells, int(geo_degree),
                                      nodes.ctypes.data, nbr.ctypes.data)
        self._chk(st, "setup_mesh")
        self.k = int(degree)
        self.n_dofs = int(self.L.hx_num_dofs(self.h))
        self.n_cells = n_cells
        return self

    def dof_coordinates(self):
        t = self.torch.empty(3, self.n_dofs, dtype=self.torch.float64, device=f"cuda:{self.device}")
        self._chk(self.L.hx_dof_coordinates(self.h, _ptr(t)), "dof_coordinates")
        return t

    def set_coefficients(self, alpha, beta, penalty: float = 2.0):
        if isinstance(alpha, np.ndarray):
            a = np.ascontiguousarray(alpha, dtype=np.float64)
            b = np.ascontiguousarray(beta, dtype=np.float64)
            st = self.L.hx_set_coefficients(self.h, a.ctypes.data, b.ctypes.data, float(penalty), 0)
        else:
            a = alpha.contiguous(); b = beta.contiguous()
            st = self.L.hx_set_coefficients(self.h, _ptr(a), _ptr(b), float(penalty), 1)
        self._chk(st, "set_coefficients")

    # -- Chebyshev preconditioner ---------------------------------------------
    def set_chebyshev(self, degree: int, lo: float, hi: float):
        self._chk(self.L.hx_set_chebyshev(self.h, int(degree), float(lo), float(hi)), "set_chebyshev")

    def estimate_eigenvalues(self, b, iters: int = 20):
        lo, hi = C.c_double(), C.c_double()
        self._chk(self.L.hx_estimate_eigenvalues(self.h, _ptr(b), int(iters), C.byref(lo), C.byref(hi)),
                  "estimate_eigenvalues")
        return lo.value, hi.value

    # -- geometric multigrid ----------------------------------------------------
    def set_multigrid(self, coarse, parent=None, octant=None):
        """Make ``coarse`` (a HelmDG on the same device and stream) the next
        coarser level: parent[f] and octant[f] per cell of this level.
        ``coarse=None`` removes the link."""
        if coarse is None:
            self._chk(self.L.hx_set_multigrid(self.h, None, None, None), "set_multigrid")
            self._mg_coarse = None
            return
        p = np.ascontiguousarray(parent, dtype=np.int32)
        o = np.ascontiguousarray(octant, dtype=np.int32)
        self._chk(self.L.hx_set_multigrid(self.h, coarse.h, p.ctypes.data, o.ctypes.data),
                  "set_multigrid")
        self._mg_coarse = coarse   # the library does not own the coarser level
        import weakref
        if not hasattr(coarse, "_mg_finer"):
            coarse._mg_finer = []
        coarse._mg_finer.append(weakref.ref(self))

    def mg_transfer(self, direction: int, x, out):
        """direction 0: out = R x (restriction); 1: out += P x (prolongation)."""
        self._chk(self.L.hx_mg_transfer(self.h, int(direction), _ptr(x), _ptr(out)), "mg_transfer")

    # -- consistent integration (2k+1 Gauss points) ----------------------------
    def set_consistent(self, alpha, beta):
        if isinstance(alpha, np.ndarray):
            a = np.ascontiguousarray(alpha, dtype=np.float64)
            b = np.ascontiguousarray(beta, dtype=np.float64)
            st = self.L.hx_set_consistent(self.h, a.ctypes.data, b.ctypes.data, 0)
        else:
            a = alpha.contiguous(); b = beta.contiguous()
            st = self.L.hx_set_consistent(self.h, _ptr(a), _ptr(b), 1)
        self._chk(st, "set_consistent")

    def apply_consistent(self, x, y=None):
        if y is None:
            y = self.torch.empty_like(x)
        self._chk(self.L.hx_apply_consistent(self.h, _ptr(x), _ptr(y)), "apply_consistent")
        return y

    # -- pressure system of an IMEX stage --------------------------------------
    def set_pressure_system(self, rho, h, gamma: float, tau: float, penalty: float = 2.0):
        if isinstance(rho, np.ndarray):
            r = np.ascontiguousarray(rho, dtype=np.float64)
            hh = np.ascontiguousarray(h, dtype=np.float64)
            st = self.L.hx_set_pressure_system(self.h, r.ctypes.data, hh.ctypes.data, float(gamma),
                                               float(tau), float(penalty), 0)
        else:
            r = rho.contiguous(); hh = h.contiguous()
            st = self.L.hx_set_pressure_system(self.h, _ptr(r), _ptr(hh), float(gamma), float(tau),
                                               float(penalty), 1)
        self._chk(st, "set_pressure_system")

    def apply_pressure_part(self, part: int, x):
        n = self.n_dofs
        shape = (3, n) if part in (HX_PS_GRAD, HX_PS_VMASS_INV) else (n,)
        y = self.torch.empty(shape, dtype=self.torch.float64, device=x.device)
        self._chk(self.L.hx_apply_pressure_part(self.h, int(part), _ptr(x), _ptr(y)),
                  "apply_pressure_part")
        return y

    def pressure_rhs(self, F, G):
        out = self.torch.empty_like(G)
        self._chk(self.L.hx_pressure_rhs(self.h, _ptr(F), _ptr(G), _ptr(out)), "pressure_rhs")
        return out

    def pressure_velocity(self, F, P):
        U = self.torch.empty_like(F)
        self._chk(self.L.hx_pressure_velocity(self.h, _ptr(F), _ptr(P), _ptr(U)), "pressure_velocity")
        return U

    def solve_pressure_fixed_point(self, rho, F, G, p, gamma: float, tau: float,
                                   params: Optional[SolveParams] = None, max_fp_iters: int = 20,
                                   fp_tol: float = 1e-10, penalty: float = 2.0, check: bool = True):
        """p (device, in/out): initial iterate, then the fixed point."""
        if params is None:
            params = default_params(method=1)
        info = SolveInfo()
        it = C.c_int(); ch = C.c_double()
        st = self.L.hx_solve_pressure_fixed_point(
            self.h, _ptr(rho), _ptr(F), _ptr(G), _ptr(p), float(gamma), float(tau), float(penalty),
            C.byref(params), int(max_fp_iters), float(fp_tol), C.byref(it), C.byref(ch),
            C.byref(info))
        if check and st not in (HX_OK, HX_ERR_NOCONV):
            self._chk(st, "solve_pressure_fixed_point")
        return p, dict(status=st, fp_iters=it.value, fp_change=ch.value, iters=info.iters,
                       true_rel_res=info.true_rel_res, ms_total=info.ms_total)

    # -- operator -------------------------------------------------------------
    def apply_operator(self, x, y=None):
        prec = HX_F64 if x.dtype == self.torch.float64 else HX_F32
        if y is None:
            y = self.torch.empty_like(x)
        self._chk(self.L.hx_apply_operator(self.h, prec, _ptr(x), _ptr(y)), "apply_operator")
        return y

    def apply_operator_part(self, part: int, x, y=None):
        """One part of A x: HX_PART_CELL (cell integrals) or HX_PART_FACE
        (face terms)."""
        prec = HX_F64 if x.dtype == self.torch.float64 else HX_F32
        if y is None:
            y = self.torch.empty_like(x)
        self._chk(self.L.hx_apply_operator_part(self.h, prec, int(part), _ptr(x), _ptr(y)),
                  "apply_operator_part")
        return y

    def set_cell_compression(self, on: bool):
        self._chk(self.L.hx_set_cell_compression(self.h, int(bool(on))), "set_cell_compression")

    def operator_info(self, prec: int = HX_F64):
        """(counts dict, algorithmic bytes of one application)."""
        counts = (C.c_int64 * 4)()
        b = C.c_double()
        self._chk(self.L.hx_operator_info(self.h, int(prec), counts, C.byref(b)), "operator_info")
        keys = ("cells", "affine_cells", "interior_faces", "affine_faces")
        return dict(zip(keys, [int(v) for v in counts])), float(b.value)

    def residual(self, b, x, r=None):
        if r is None:
            r = self.torch.empty_like(b)
        self._chk(self.L.hx_residual(self.h, _ptr(b), _ptr(x), _ptr(r)), "residual")
        return r

    def apply_preconditioner(self, r, z=None, kind: int = HX_PC_BLOCK_JACOBI):
        prec = HX_F64 if r.dtype == self.torch.float64 else HX_F32
        if z is None:
            z = self.torch.empty_like(r)
        self._chk(self.L.hx_apply_preconditioner(self.h, kind, prec, _ptr(r), _ptr(z)),
                  "apply_preconditioner")
        return z

    def solve(self, b, x=None, params: Optional[SolveParams] = None, history: int = 0,
              check: bool = True):
        if params is None:
            params = default_params()
        if x is None:
            x = self.torch.zeros_like(b)
        info = SolveInfo()
        hist = None
        if history:
            hist = (C.c_double * history)()
            info.history = C.cast(hist, C.POINTER(C.c_double))
            info.history_len = history
        st = self.L.hx_solve(self.h, C.byref(params), _ptr(b), _ptr(x), C.byref(info))
        if check and st not in (HX_OK, HX_FALLBACK_USED, HX_ERR_NOCONV):
            self._chk(st, "solve")
        res = dict(status=st, iters=info.iters, restarts=info.restarts,
                   fallback_used=bool(info.fallback_used), inner_iters=info.inner_iters,
                   true_rel_res=info.true_rel_res, ms_total=info.ms_total, ms_op=info.ms_op,
                   ms_pc=info.ms_pc, ms_orth=info.ms_orth)
        if hist is not None:
            res["history"] = list(hist[:info.history_len])
        return x, res

    def dot(self, x, y) -> float:
        out = C.c_double()
        self._chk(self.L.hx_dot(self.h, x.numel(), _ptr(x), _ptr(y), C.byref(out)), "dot")
        return out.value

    # -- learned preconditioner -------------------------------------------
    def network_size(self) -> int:
        return int(self.L.hx_network_size(self.h))

    def set_network(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        self._chk(self.L.hx_set_network(self.h, w.ctypes.data, w.size), "set_network")

    def get_network(self) -> np.ndarray:
        w = np.zeros(self.network_size(), dtype=np.float32)
        self._chk(self.L.hx_get_network(self.h, w.ctypes.data, w.size), "get_network")
        return w

    def n_features(self) -> int:
        n = self.k + 1
        return n ** 3 + 6 * n * n + 1

    def gather_features(self, r):
        F = self.torch.empty(self.n_cells, self.n_features(), dtype=self.torch.float32,
                             device=r.device)
        s = self.torch.empty(self.n_cells, dtype=self.torch.float32, device=r.device)
        self._chk(self.L.hx_gather_features(self.h, _ptr(r), _ptr(F), _ptr(s)), "gather_features")
        return F, s

    def training_pair(self, b, x_star, x_j, clip: float = 0.0):
        """Per-cell features and residual-learning targets from a solver
        iterate (targets limited to [-clip, clip] when clip > 0)."""
        F = self.torch.empty(self.n_cells, self.n_features(), dtype=self.torch.float32,
                             device=b.device)
        T = self.torch.empty(self.n_cells, (self.k + 1) ** 3, dtype=self.torch.float32,
                             device=b.device)
        self._chk(self.L.hx_training_pair(self.h, _ptr(b), _ptr(x_star), _ptr(x_j), float(clip), _ptr(F),
                                          _ptr(T)), "training_pair")
        return F, T

    def network_forward(self, feats):
        n_out = (self.k + 1) ** 3
        out = self.torch.empty(feats.shape[0], n_out, dtype=self.torch.float32, device=feats.device)
        self._chk(self.L.hx_network_forward(self.h, _ptr(feats), feats.shape[0], _ptr(out)),
                  "network_forward")
        return out


    def network_forward_noalloc(self, feats, out=None):
        """The same forward pass with the library's static work buffers (no
        device allocation inside the call); ``out`` may be given."""
        n_out = (self.k + 1) ** 3
        if out is None:
            out = self.torch.empty(feats.shape[0], n_out, dtype=self.torch.float32,
                                   device=feats.device)
        self._chk(self.L.hx_network_forward_noalloc(self.h, _ptr(feats), feats.shape[0], _ptr(out)),
                  "network_forward_noalloc")
        return out

    def network_noalloc_max_batch(self) -> int:
        return int(self.L.hx_network_noalloc_max_batch(self.h))
    def train_step(self, feats, targets, lr: float, want_grad: bool = False,
                   want_loss: bool = True):
        loss = C.c_float()
        g = None
        if want_grad:
            g = self.torch.empty(self.network_size(), dtype=self.torch.float32, device=feats.device)
        self._chk(self.L.hx_train_step(self.h, _ptr(feats), _ptr(targets), feats.shape[0],
                                       float(lr), C.byref(loss) if want_loss else None,
                                       _ptr(g) if g is not None else None),
                  "train_step")
        return (loss.value if want_loss else None), g

    def network_trace(self, what: int, batch: int) -> np.ndarray:
        """One intermediate of the last train_step (HX_TRACE_*), [batch, width]."""
        n, hid = self.k + 1, 256
        width = {HX_TRACE_INPUT: n ** 3 + 6 * n * n + 1, HX_TRACE_OUT: n ** 3,
                 HX_TRACE_DOUT: n ** 3}.get(what, hid)
        out = np.zeros((batch, width), dtype=np.float32)
        self._chk(self.L.hx_network_trace(self.h, what, out.ctypes.data, out.size), "network_trace")
        return out

    def debug_export(self, what: int, shape, dtype=np.float64) -> np.ndarray:
        out = np.zeros(shape, dtype=dtype)
        self._chk(self.L.hx_debug_export(self.h, what, out.ctypes.data, out.nbytes), "debug_export")
        return out


__all__ = ["HelmDG", "HXError", "SolveParams", "SolveInfo", "default_params", "load"] + \
    [n for n in list(globals()) if n.startswith("HX_")]
