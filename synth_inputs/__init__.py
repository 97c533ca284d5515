"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module holds no arithmetic of the discretisation: it only produces
meshes (geometry nodes at equispaced reference points plus a face-neighbour
table), analytic coefficient and right-hand-side fields as plain functions of
physical position, and seeded random numbers (vectors, network weights).
Whoever needs those fields at the degrees of freedom evaluates the functions at
coordinates they computed themselves.

Mesh format (the input of ``setup_mesh``):

* ``nodes``: float64 ``[n_cells, (g+1)**3, 3]``; node ``a + (g+1)*b + (g+1)**2*c``
  is the image of the reference point ``(a/g, b/g, c/g)`` of the unit cube, so
  the cell map is the tensor-product Lagrange interpolant of degree ``g``
  through equispaced nodes.
* ``nbr``: int64 ``[n_cells, 6]`` with the neighbour across the
  ``-x, +x, -y, +y, -z, +z`` faces, ``-1`` on a (natural Neumann) boundary.
  Meshes are conforming with standard orientation: the ``+d`` face of a cell
  is the ``-d`` face of its ``+d`` neighbour.
* cell index ``cx + nx*(cy + ny*cz)``.

Random draws use ``numpy.random.default_rng(seed)`` (PCG64) in the order
documented at each function.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, Optional, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# meshes
# ---------------------------------------------------------------------------


@dataclass
class Mesh:
    nodes: np.ndarray            # [n_cells, (g+1)^3, 3] float64
    nbr: np.ndarray              # [n_cells, 6] int64
    g: int
    dims: Tuple[int, int, int]
    lo: Tuple[float, float, float]
    hi: Tuple[float, float, float]
    periodic: Tuple[bool, bool, bool]
    name: str = ""
    meta: dict = field(default_factory=dict)
    hang: Optional[np.ndarray] = None   # [n, 4] non-conforming quarter faces (see refined_mesh)

    @property
    def n_cells(self) -> int:
        return int(self.nbr.shape[0])


def box_neighbours(nx: int, ny: int, nz: int,
                   periodic=(False, False, False)) -> np.ndarray:
    """Face-neighbour table of a structured nx*ny*nz block (x fastest)."""
    cx, cy, cz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz),
                             indexing="ij")
    cx = cx.transpose(2, 1, 0).ravel()
    cy = cy.transpose(2, 1, 0).ravel()
    cz = cz.transpose(2, 1, 0).ravel()
    dims = (nx, ny, nz)
    coords = [cx, cy, cz]
    nbr = np.empty((nx * ny * nz, 6), dtype=np.int64)
    for d in range(3):
        for s, step in enumerate((-1, 1)):
            c = [a.copy() for a in coords]
            c[d] = c[d] + step
            out = (c[d] < 0) | (c[d] >= dims[d])
            if periodic[d]:
                c[d] = np.mod(c[d], dims[d])
                idx = c[0] + nx * (c[1] + ny * c[2])
            else:
                cc = np.clip(c[d], 0, dims[d] - 1)
                c[d] = cc
                idx = c[0] + nx * (c[1] + ny * c[2])
                idx = np.where(out, -1, idx)
            nbr[:, 2 * d + s] = idx
    return nbr


def box_mesh(nx: int, ny: int, nz: int,
             lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
             periodic=(True, True, True), g: int = 1,
             mapping: Optional[Callable] = None, name: str = "box") -> Mesh:
    """Structured hexahedral mesh of a box, optionally deformed.

    ``mapping(x, y, z) -> (x', y', z')`` acts on the physical positions of the
    equispaced geometry nodes of every cell (vectorised numpy arrays).
    """
    if g < 1:
        raise ValueError("geometry degree must be >= 1")
    lo = tuple(float(v) for v in lo)
    hi = tuple(float(v) for v in hi)
    h = [(hi[d] - lo[d]) / n for d, n in enumerate((nx, ny, nz))]
    t = np.arange(g + 1, dtype=np.float64) / g
    # reference node offsets, node index a + (g+1) b + (g+1)^2 c
    ta = np.tile(t, (g + 1) ** 2)
    tb = np.tile(np.repeat(t, g + 1), g + 1)
    tc = np.repeat(t, (g + 1) ** 2)
    n_cells = nx * ny * nz
    cidx = np.arange(n_cells, dtype=np.int64)
    cx = (cidx % nx).astype(np.float64)
    cy = ((cidx // nx) % ny).astype(np.float64)
    cz = (cidx // (nx * ny)).astype(np.float64)
    nodes = np.empty((n_cells, (g + 1) ** 3, 3), dtype=np.float64)
    X = lo[0] + (cx[:, None] + ta[None, :]) * h[0]
    Y = lo[1] + (cy[:, None] + tb[None, :]) * h[1]
    Z = lo[2] + (cz[:, None] + tc[None, :]) * h[2]
    if mapping is not None:
        X, Y, Z = mapping(X, Y, Z)
    nodes[:, :, 0] = X
    nodes[:, :, 1] = Y
    nodes[:, :, 2] = Z
    nbr = box_neighbours(nx, ny, nz, periodic)
    return Mesh(nodes=nodes, nbr=nbr, g=g, dims=(nx, ny, nz), lo=lo, hi=hi,
                periodic=tuple(bool(p) for p in periodic), name=name)


def refined_mesh(nx: int, ny: int, nz: int, region, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                 periodic=(True, True, True), g: int = 1, mapping: Optional[Callable] = None,
                 name: str = "refined") -> Mesh:
    """A structured nx*ny*nz mesh whose coarse cells with indices in
    ``region`` = ((i0, i1), (j0, j1), (l0, l1)) (half-open) are split into
    2x2x2 children: a non-conforming mesh with 2:1 faces.

    Cells: the unrefined coarse cells (x fastest), then the children in the
    order of the fine grid (x fastest).  Every cell's geometry nodes are the
    (mapped) images of its own equispaced reference nodes.  Faces between two
    cells of the same size are conforming; a face between a child and an
    unrefined coarse cell is marked -2 in ``nbr`` on both sides and listed in
    ``hang`` as {coarse cell, its face, fine cell, quarter s}: face (f ^ 1) of
    the fine cell is quarter s = s1 + 2 s2 of face f of the coarse cell, s1
    (s2) the half along the first (second) of the two tangential directions."""
    if g < 1:
        raise ValueError("geometry degree must be >= 1")
    dims = (nx, ny, nz)
    ref = np.zeros(dims, dtype=bool)
    (i0, i1), (j0, j1), (l0, l1) = region
    ref[i0:i1, j0:j1, l0:l1] = True
    h = [(hi[d] - lo[d]) / dims[d] for d in range(3)]
    cid = -np.ones(dims, dtype=np.int64)
    cells = []                         # (origin, size, level, position)
    for cz in range(nz):
        for cy in range(ny):
            for cx in range(nx):
                if not ref[cx, cy, cz]:
                    cid[cx, cy, cz] = len(cells)
                    cells.append(((lo[0] + cx * h[0], lo[1] + cy * h[1], lo[2] + cz * h[2]),
                                  tuple(h), 0, (cx, cy, cz)))
    fdims = tuple(2 * v for v in dims)
    fid = -np.ones(fdims, dtype=np.int64)
    for fz in range(fdims[2]):
        for fy in range(fdims[1]):
            for fx in range(fdims[0]):
                if ref[fx // 2, fy // 2, fz // 2]:
                    fid[fx, fy, fz] = len(cells)
                    cells.append(((lo[0] + fx * h[0] / 2, lo[1] + fy * h[1] / 2, lo[2] + fz * h[2] / 2),
                                  tuple(v / 2 for v in h), 1, (fx, fy, fz)))
    n_cells = len(cells)
    t = np.arange(g + 1, dtype=np.float64) / g
    ta = np.tile(t, (g + 1) ** 2)
    tb = np.tile(np.repeat(t, g + 1), g + 1)
    tc = np.repeat(t, (g + 1) ** 2)
    org = np.array([c[0] for c in cells])
    siz = np.array([c[1] for c in cells])
    X = org[:, 0:1] + ta[None, :] * siz[:, 0:1]
    Y = org[:, 1:2] + tb[None, :] * siz[:, 1:2]
    Z = org[:, 2:3] + tc[None, :] * siz[:, 2:3]
    if mapping is not None:
        X, Y, Z = mapping(X, Y, Z)
    nodes = np.stack([X, Y, Z], axis=-1)
    nbr = np.empty((n_cells, 6), dtype=np.int64)
    hang = []
    for c, (_, _, level, pos) in enumerate(cells):
        gdims = dims if level == 0 else fdims
        for d in range(3):
            t1, t2 = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
            for s, step in enumerate((-1, 1)):
                f = 2 * d + s
                q = list(pos)
                q[d] += step
                if q[d] < 0 or q[d] >= gdims[d]:
                    if not periodic[d]:
                        nbr[c, f] = -1
                        continue
                    q[d] %= gdims[d]
                if level == 0:
                    if ref[tuple(q)]:
                        nbr[c, f] = -2          # four fine cells: recorded from their side
                    else:
                        nbr[c, f] = cid[tuple(q)]
                else:
                    parent = tuple(v // 2 for v in q)
                    if ref[parent]:
                        nbr[c, f] = fid[tuple(q)]
                    else:
                        nbr[c, f] = -2
                        quarter = (pos[t1] % 2) + 2 * (pos[t2] % 2)
                        hang.append((cid[parent], f ^ 1, c, quarter))
    return Mesh(nodes=nodes, nbr=nbr, g=g, dims=dims, lo=tuple(lo), hi=tuple(hi),
                periodic=tuple(bool(p) for p in periodic), name=name,
                hang=np.array(hang, dtype=np.int64).reshape(-1, 4))


def refined_terrain_mesh(nx: int = 16, ny: int = 4, nz: int = 8, g: int = 4, region=None) -> Mesh:
    """The terrain channel with the cells above the ridge refined once (a
    non-conforming mesh: the paper's second mesh refines around the hill).
    Default region: the middle half in x, all of y, the bottom half in z."""
    T = TERRAIN
    if region is None:
        region = ((nx // 4, 3 * nx // 4), (0, ny), (0, max(1, nz // 2)))
    return refined_mesh(nx, ny, nz, region, lo=(-T["Lx"] / 2, 0.0, 0.0),
                        hi=(T["Lx"] / 2, T["Ly"], T["Lz"]), periodic=(True, True, False), g=g,
                        mapping=terrain_mapping, name=f"terrain-refined-{nx}x{ny}x{nz}")


# --- the workloads -------------------------------------------------------

#: isothermal background and time-step scaling of the terrain workloads
TERRAIN = dict(Lx=40000.0, Ly=10000.0, Lz=20000.0, h0=400.0, a=2000.0,
               H=7300.0, c=340.0, dt=1.0)


def ridge_height(x):
    """Gaussian ridge h(x) = 400 m * exp(-(x / 2 km)^2)."""
    return TERRAIN["h0"] * np.exp(-(x / TERRAIN["a"]) ** 2)


def terrain_mapping(x, y, z):
    """Terrain-following map z' = z + h(x) (1 - z / Z_top) (decays linearly)."""
    Lz = TERRAIN["Lz"]
    return x, y, z + ridge_height(x) * (1.0 - z / Lz)


def cube_mesh(n: int = 4, g: int = 1, periodic=(True, True, True)) -> Mesh:
    """Unit cube [0,1]^3 with n^3 affine cells (periodic by default)."""
    return box_mesh(n, n, n, periodic=periodic, g=g, name=f"cube{n}")


def terrain_mesh(nx: int = 32, ny: int = 8, nz: int = 16, g: int = 4) -> Mesh:
    """Terrain-following channel, x in [-20, 20] km and y in [0, 10] km
    periodic, zeta in [0, 20] km with Neumann bottom and top, ridge in x."""
    T = TERRAIN
    m = box_mesh(nx, ny, nz, lo=(-T["Lx"] / 2, 0.0, 0.0),
                 hi=(T["Lx"] / 2, T["Ly"], T["Lz"]),
                 periodic=(True, True, False), g=g, mapping=terrain_mapping,
                 name=f"terrain{nx}x{ny}x{nz}")
    return m


def refinement_parents(nx: int, ny: int, nz: int):
    """Cell map of the box mesh (2nx, 2ny, 2nz) to the box mesh (nx, ny, nz)
    over the same box: for each fine cell its parent cell and the octant
    ox + 2 oy + 4 oz it occupies (cells numbered x fastest, then y, then z,
    both meshes with the same axis orientation)."""
    f = np.arange(8 * nx * ny * nz, dtype=np.int64)
    fx, fy, fz = f % (2 * nx), (f // (2 * nx)) % (2 * ny), f // (4 * nx * ny)
    parent = fx // 2 + nx * (fy // 2 + ny * (fz // 2))
    octant = (fx & 1) + 2 * (fy & 1) + 4 * (fz & 1)
    return parent.astype(np.int32), octant.astype(np.int32)


def wavy_mapping(eps: float = 0.04):
    """A smooth, fully periodic deformation of the unit cube (curved cells)."""
    tp = 2.0 * math.pi

    def f(x, y, z):
        return (x + eps * np.sin(tp * y) * np.sin(tp * z),
                y + eps * np.sin(tp * z) * np.sin(tp * x),
                z + eps * np.sin(tp * x) * np.sin(tp * y))
    return f


def wavy_cube_mesh(n: int, g: int, eps: float = 0.04,
                   periodic=(True, True, True)) -> Mesh:
    return box_mesh(n, n, n, periodic=periodic, g=g, mapping=wavy_mapping(eps),
                    name=f"wavy{n}")


def random_affine_mapping(seed: int, amp: float = 0.1):
    """A random affine map (shear + stretch) with positive determinant.

    Draws: one 3x3 matrix of U[-amp, amp] entries."""
    rng = np.random.default_rng(seed)
    A = np.eye(3) + rng.uniform(-amp, amp, size=(3, 3))

    def f(x, y, z):
        return (A[0, 0] * x + A[0, 1] * y + A[0, 2] * z,
                A[1, 0] * x + A[1, 1] * y + A[1, 2] * z,
                A[2, 0] * x + A[2, 1] * y + A[2, 2] * z)
    return f


def random_node_jitter(mesh: Mesh, seed: int, amp: float) -> Mesh:
    """Displace every geometry node by an independent U[-amp, amp]^3 draw,
    consistently across shared faces (nodes are keyed by position) -- only for
    non-periodic meshes, where shared positions coincide exactly."""
    if any(mesh.periodic):
        raise ValueError("jitter only for non-periodic meshes")
    rng = np.random.default_rng(seed)
    flat = mesh.nodes.reshape(-1, 3)
    key = np.round(flat * 1e9).astype(np.int64)
    uniq, inv = np.unique(key, axis=0, return_inverse=True)
    disp = rng.uniform(-amp, amp, size=(uniq.shape[0], 3))
    nodes = (flat + disp[inv.ravel()]).reshape(mesh.nodes.shape)
    return Mesh(nodes=nodes, nbr=mesh.nbr.copy(), g=mesh.g, dims=mesh.dims,
                lo=mesh.lo, hi=mesh.hi, periodic=mesh.periodic,
                name=mesh.name + "-jitter")


# ---------------------------------------------------------------------------
# coefficient fields (functions of physical position)
# ---------------------------------------------------------------------------

def const_coefficients(alpha: float = 1.0, beta: float = 0.01):
    """Constant alpha and beta (the periodic-cube workload uses 1 and 0.01)."""
    def a(x, y, z):
        return np.full_like(np.asarray(x, dtype=np.float64), alpha)

    def b(x, y, z):
        return np.full_like(np.asarray(x, dtype=np.float64), beta)
    return a, b


def terrain_coefficients():
    """Isothermal hydrostatic background: alpha = rho0/rho(z) = exp(z/H),
    beta = (c dt)^2 exp(z/H)."""
    T = TERRAIN
    tau = (T["c"] * T["dt"]) ** 2

    def a(x, y, z):
        return np.exp(np.asarray(z, dtype=np.float64) / T["H"])

    def b(x, y, z):
        return tau * np.exp(np.asarray(z, dtype=np.float64) / T["H"])
    return a, b


def terrain_pressure_fields(gamma: float = 1.4):
    """Fields of the pressure system on the isothermal background: density
    ratio rho/rho0 = exp(-z/H) and the specific enthalpy of an isothermal
    ideal gas, h = c^2/(gamma - 1) (constant), as functions of (x, y, z)."""
    T = TERRAIN

    def rho(x, y, z):
        return np.exp(-np.asarray(z, dtype=np.float64) / T["H"])

    def h(x, y, z):
        return np.full_like(np.asarray(x, dtype=np.float64), T["c"] ** 2 / (gamma - 1.0))
    return rho, h


def random_smooth_coefficients(seed: int, lo=0.5, hi=2.0, scale=1.0):
    """Smooth positive fields: lo + (hi-lo) * (1 + sin(...)) / 2, random phases.

    Draws: 6 phases U[0, 2 pi) then 6 integer wavenumbers in {1, 2}."""
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2.0 * math.pi, 6)
    kk = rng.integers(1, 3, 6)
    tp = 2.0 * math.pi

    def fa(x, y, z):
        s = np.sin(tp * kk[0] * x + ph[0]) * np.cos(tp * kk[1] * y + ph[1]) \
            * np.cos(tp * kk[2] * z + ph[2])
        return lo + (hi - lo) * 0.5 * (1.0 + s)

    def fb(x, y, z):
        s = np.cos(tp * kk[3] * x + ph[3]) * np.sin(tp * kk[4] * y + ph[4]) \
            * np.cos(tp * kk[5] * z + ph[5])
        return scale * (lo + (hi - lo) * 0.5 * (1.0 + s))
    return fa, fb


# ---------------------------------------------------------------------------
# right-hand sides
# ---------------------------------------------------------------------------

def rhs_cube(seed: int):
    """f(x) = sum_m a_m cos(2 pi kappa_m . x + phi_m), m = 1..5, on the unit cube.

    Draws, in order: a (5 x N(0,1)); kappa (5 x 3 integers in {-2..2}, a zero
    vector is redrawn); phi (5 x U[0, 2 pi))."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=5)
    kap = rng.integers(-2, 3, size=(5, 3))
    for m in range(5):
        while not kap[m].any():
            kap[m] = rng.integers(-2, 3, size=3)
    phi = rng.uniform(0.0, 2.0 * math.pi, 5)
    tp = 2.0 * math.pi

    def f(x, y, z):
        out = np.zeros_like(np.asarray(x, dtype=np.float64))
        for m in range(5):
            out += a[m] * np.cos(tp * (kap[m, 0] * x + kap[m, 1] * y
                                       + kap[m, 2] * z) + phi[m])
        return out
    return f


def rhs_terrain(seed: int):
    """5 modes periodic in (x, y) on the channel, cos(pi m_z z / Z_top) in z.

    Draws, in order: a (5 x N(0,1)); (m_x, m_y) (5 x 2 integers in {-2..2});
    m_z (5 integers in {0, 1, 2}); phi (5 x U[0, 2 pi))."""
    T = TERRAIN
    rng = np.random.default_rng(seed)
    a = rng.normal(size=5)
    mxy = rng.integers(-2, 3, size=(5, 2))
    mz = rng.integers(0, 3, size=5)
    phi = rng.uniform(0.0, 2.0 * math.pi, 5)
    tp = 2.0 * math.pi

    def f(x, y, z):
        out = np.zeros_like(np.asarray(x, dtype=np.float64))
        for m in range(5):
            out += a[m] * np.cos(tp * (mxy[m, 0] * (x + T["Lx"] / 2) / T["Lx"]
                                       + mxy[m, 1] * y / T["Ly"]) + phi[m]) \
                * np.cos(math.pi * mz[m] * z / T["Lz"])
        return out
    return f


def random_vector(n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """n draws of N(0,1)."""
    return np.random.default_rng(seed).normal(size=n).astype(dtype)


# ---------------------------------------------------------------------------
# network parameters of the learned preconditioner
# ---------------------------------------------------------------------------

def mlp_layer_sizes(n_in: int = 276, hidden: int = 256, n_out: int = 125):
    return [(hidden, n_in), (hidden, hidden), (n_out, hidden)]


def mlp_param_count(n_in: int = 276, hidden: int = 256, n_out: int = 125) -> int:
    return sum(o * i + o for o, i in mlp_layer_sizes(n_in, hidden, n_out))


def mlp_init(seed: int, n_in: int = 276, hidden: int = 256, n_out: int = 125,
             out_scale: float = 1.0) -> np.ndarray:
    """Flat float32 parameter vector [W1, b1, W2, b2, W3, b3] (W row-major
    [out, in]).  W_l ~ U[-sqrt(6/in), sqrt(6/in)] (He-uniform), biases 0;
    the last layer is multiplied by ``out_scale``.  Draws: W1, W2, W3 in order."""
    rng = np.random.default_rng(seed)
    parts = []
    layers = mlp_layer_sizes(n_in, hidden, n_out)
    for li, (o, i) in enumerate(layers):
        lim = math.sqrt(6.0 / i)
        w = rng.uniform(-lim, lim, size=(o, i))
        if li == len(layers) - 1:
            w = w * out_scale
        parts.append(w.ravel())
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)
