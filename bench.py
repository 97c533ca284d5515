"""Benchmark of the DG Helmholtz pressure operator and solve on one MI355X.

Timed step: one application of the fused cell + face operator (y = A x, FP64)
on the terrain-following channel with 256 x 64 x 64 Q4 cells (131,072,000
dofs), inputs resident in HBM.  ``value`` is GDoF/s = n_dofs / (time per
application).  The JSON line also carries

* ``roofline``: algorithmic bytes per application (105.6 B/dof: x and y,
  7 merged cell values and 3 x 7 x 25 / 125 merged face values per dof, FP64)
  over the event-timed kernel duration, against the 8 TB/s HBM peak, and the
  HBM traffic measured by rocprofv3 counters (from the committed profile, null
  if the kernel source changed since);
* ``solve``: time to a 1e-8 relative true residual for plain FP64 (FGMRES and
  CG with block Jacobi, CG with the paper's Helmholtz and internal-energy
  diagonal preconditioners), mixed precision and learned forms;
* ``cpu_baseline``: the FP64 oracle timed on the host cores on a sample of the
  same workload.

Usage: python bench.py [--gpus 1] [--steps 50] [--warmup 5]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

def alg_bytes_per_dof(k: int) -> float:
    """FP64 bytes per dof of the general data layout: x and y (16), the merged
    cell data (7 values per Gauss point = per dof, 56) and the merged face data
    (3 faces x 7 values x (k+1)^2 points per cell, 168/(k+1)); 105.6 at k = 4.
    The library's own byte model (hx_operator_info) counts interior faces
    only and the compressed data of affine cells."""
    return 16.0 + 56.0 + 3 * 7 * 8.0 / (k + 1)
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "op_apply_f64_terrain256x64x64_k4_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2505_00384_amd", "csrc", "operator.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def read_traffic(n_dofs: int):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source."""
    if not os.path.exists(PROFILE_TRAFFIC):
        return None
    kv = {}
    for line in open(PROFILE_TRAFFIC):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("operator_source_sha256_16") != kernel_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def setup(ctx_cls, mesh, k, torch, dev, timing=None):
    """Mesh and coefficients on the device; with ``timing`` (a dict) also the
    wall time of setup_mesh and of one more set_coefficients call (the step
    the paper's solver repeats at every fixed-point iteration)."""
    from synth_inputs import terrain_coefficients
    ctx = ctx_cls(0)
    t0 = time.time()
    ctx.setup_mesh(k, mesh.nodes, mesh.nbr, mesh.g, hang=getattr(mesh, "hang", None))
    torch.cuda.synchronize()
    t1 = time.time()
    xyz = ctx.dof_coordinates()
    fa, fb = terrain_coefficients()
    a, b = field_on_device(fa, xyz, torch), field_on_device(fb, xyz, torch)
    ctx.set_coefficients(a, b, 2.0)
    torch.cuda.synchronize()
    t_all = time.time() - t0
    if timing is not None:
        t2 = time.time()
        ctx.set_coefficients(a, b, 2.0)
        torch.cuda.synchronize()
        timing.update(setup_mesh_s=round(t1 - t0, 3),
                      set_coefficients_ms=round((time.time() - t2) * 1e3, 2))
    return ctx, xyz, t_all


def rhs_on_device(xyz, seed, torch):
    from synth_inputs import rhs_terrain
    return field_on_device(rhs_terrain(seed), xyz, torch)


def field_on_device(f, xyz, torch):
    """Evaluate an analytic input field (numpy function of x, y, z) at the
    library's dof coordinates, in chunks on the host, and upload it."""
    x = xyz.cpu().numpy()
    out = np.empty(x.shape[1])
    step = 1 << 24
    for s in range(0, x.shape[1], step):
        out[s:s + step] = f(x[0, s:s + step], x[1, s:s + step], x[2, s:s + step])
    return torch.from_numpy(out).to(xyz.device)


def time_matvec(ctx, x, y, steps, warmup, torch, part=0):
    """Event-timed average of `steps` back-to-back applications on the
    context's stream (torch's current stream), after `warmup` untimed ones."""
    def launch():
        if part:
            ctx.apply_operator_part(part, x, y)
        else:
            ctx.apply_operator(x, y)
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        launch()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps        # ms per application


def median_windows(ctx, x, y, torch, windows=5, launches=100, part=0):
    """Median over `windows` timing windows of `launches` applications each."""
    t = sorted(time_matvec(ctx, x, y, launches, 2, torch, part) for _ in range(windows))
    return t[len(t) // 2], t


def operator_windows(hx, ctx, x, y, torch, n, op_bytes, counts):
    """Median of 5 windows of 100 applications, the cell and face parts
    alone, and the general data layout (compression off) for comparison."""
    med, wins = median_windows(ctx, x, y, torch)
    t_cell, _ = median_windows(ctx, x, y, torch, windows=3, launches=50, part=hx.HX_PART_CELL)
    t_face, _ = median_windows(ctx, x, y, torch, windows=3, launches=50, part=hx.HX_PART_FACE)
    ctx.set_cell_compression(False)
    _, gen_bytes = ctx.operator_info(hx.HX_F64)
    t_gen, _ = median_windows(ctx, x, y, torch, windows=3, launches=50)
    ctx.set_cell_compression(True)
    return dict(
        bytes_per_dof=round(op_bytes / n, 2), counts=counts,
        median_of_5x100_ms=round(med, 4), windows_ms=[round(v, 4) for v in wins],
        cell_part_ms=round(t_cell, 4), face_part_ms=round(t_face, 4),
        general_data_ms=round(t_gen, 4), general_bytes_per_dof=round(gen_bytes / n, 2),
        general_data_frac=round(gen_bytes / (t_gen * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))


def nonconforming_suite(hx, torch, dev, k):
    """The 32x8x16 terrain channel with the cells over the ridge refined once
    (the middle half in x, the bottom half in z: a non-conforming mesh with
    2:1 faces, like the paper's second mesh around its hill): the operator,
    and CG / FGMRES to 1e-8 with block Jacobi and with the paper's two
    diagonal preconditioners (section 3.1: the Helmholtz one, the inverse
    diagonal of the volume terms, against the internal-energy one, the
    inverse mass diagonal)."""
    import synth_inputs as si
    m = si.refined_terrain_mesh(32, 8, 16, g=4)
    ctx, xyz, _ = setup(hx.HelmDG, m, k, torch, dev)
    b = rhs_on_device(xyz, 0, torch)
    del xyz
    y = torch.empty_like(b)
    ms = time_matvec(ctx, b, y, 50, 5, torch)
    counts, op_bytes = ctx.operator_info(hx.HX_F64)
    out = dict(cells=m.n_cells, quarter_faces=int(m.hang.shape[0]), n_dofs=ctx.n_dofs,
               matvec_ms=round(ms, 4), gdofs=round(ctx.n_dofs / (ms * 1e-3) / 1e9, 3),
               bytes_per_dof=round(op_bytes / ctx.n_dofs, 2))
    out["solve"] = solve_suite(hx, ctx, b, torch, [
        ("fp64_cg_bj", hx.default_params(method=0, rtol=1e-8)),
        ("fp64_cg_helmholtz_diag", hx.default_params(method=0, rtol=1e-8, max_iter=20000,
                                                     pc=hx.HX_PC_HELMHOLTZ_DIAG)),
        ("fp64_cg_mass_diag", hx.default_params(method=0, rtol=1e-8, max_iter=20000,
                                                pc=hx.HX_PC_MASS_DIAG)),
        ("fp64_fgmres_helmholtz_diag", hx.default_params(method=1, restart=30, rtol=1e-8,
                                                         max_iter=20000, pc=hx.HX_PC_HELMHOLTZ_DIAG)),
        ("fp64_fgmres_mass_diag", hx.default_params(method=1, restart=30, rtol=1e-8,
                                                    max_iter=20000, pc=hx.HX_PC_MASS_DIAG)),
        ("mixed_fp32_inner", hx.default_params(method=1, restart=10, rtol=1e-8, mixed=1,
                                               inner_iters=32))], "nonconforming")
    ctx.close()
    return out


def solve_suite(hx, ctx, b, torch, forms, label, keep=None):
    """Time each solve form; with ``keep`` (a dict) the solutions are kept on
    the host, by form name, for the oracle comparison of the CPU leg."""
    out = {}
    for name, params in forms:
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.time()
        x, info = ctx.solve(b, x, params)
        torch.cuda.synchronize()
        wall = (time.time() - t0) * 1e3
        if keep is not None:
            keep[name] = x.cpu().numpy()
        out[name] = dict(ms=round(wall, 3), iters=info["iters"], inner_iters=info["inner_iters"],
                         true_rel_res=info["true_rel_res"], status=hx.STATUS_NAMES[info["status"]],
                         ms_op=round(info["ms_op"], 3), ms_pc=round(info["ms_pc"], 3),
                         ms_orth=round(info["ms_orth"], 3))
        log(f"{label} {name}: {out[name]}")
    return out


def multigrid_suite(hx, ctx, b, torch, dev, dims, k, fine_bounds, levels=5, smooth_degree=2,
                    smooth_ratio=15.0, coarse_degree=12, consistent=False):
    """CG with one geometric-multigrid V-cycle per iteration: the terrain
    channel coarsened by two in every direction down to `levels` levels, each
    level's operator re-discretised with the coefficients at its own dofs,
    Chebyshev smoothing of degree 2 on [1.1 hi / 15, 1.1 hi] of each level's
    Lanczos range (20 steps on a random vector) and a degree-12 polynomial
    over the whole range on the coarsest level.  The set-up of the coarse
    levels and their estimates is timed apart from the solve.  With
    ``consistent`` the system with consistent integration (set on ctx) is
    solved too, preconditioned by the same cycle of the fast operator."""
    import synth_inputs as si
    nx, ny, nz = dims
    torch.cuda.synchronize()
    t0 = time.time()
    ctxs, maps = [ctx], []
    for l in range(1, levels):
        s = 2 ** l
        if nx % s or ny % s or nz % s:
            break
        m = si.terrain_mesh(nx // s, ny // s, nz // s, g=4)
        c, xyz, _ = setup(hx.HelmDG, m, k, torch, dev)
        del xyz
        ctxs.append(c)
        maps.append(si.refinement_parents(nx // s, ny // s, nz // s))
    gen = torch.Generator(device=dev)
    bounds = [fine_bounds]
    for l, c in enumerate(ctxs[1:], start=1):
        gen.manual_seed(10 + l)
        rv = torch.randn(c.n_dofs, dtype=torch.float64, device=dev, generator=gen)
        bounds.append(c.estimate_eigenvalues(rv, 20))
        del rv
    for l, c in enumerate(ctxs):
        lo, hi = bounds[l]
        if l + 1 < len(ctxs):
            c.set_chebyshev(smooth_degree, 1.1 * hi / smooth_ratio, 1.1 * hi)
            c.set_multigrid(ctxs[l + 1], *maps[l])
        else:
            c.set_chebyshev(coarse_degree, 0.9 * lo, 1.1 * hi)
    torch.cuda.synchronize()
    t_setup = time.time() - t0
    out = solve_suite(hx, ctx, b, torch, [
        ("fp64_cg_multigrid", hx.default_params(method=0, rtol=1e-8, pc=hx.HX_PC_MULTIGRID)),
        ("fp64_cg_multigrid_fp32_cycle", hx.default_params(method=0, rtol=1e-8,
                                                           pc=hx.HX_PC_MULTIGRID_MIXED))]
        + ([("consistent_cg_multigrid_fp32_cycle", hx.default_params(
            method=0, rtol=1e-8, system=2, pc=hx.HX_PC_MULTIGRID_MIXED))] if consistent else []),
        "C3")
    for name in out:
        out[name].update(
            levels=[f"{nx // 2 ** l}x{ny // 2 ** l}x{nz // 2 ** l}" for l in range(len(ctxs))],
            smoother=f"chebyshev{smooth_degree} [hi/{smooth_ratio:g}, 1.1 hi]",
            coarse=f"chebyshev{coarse_degree} [0.9 lo, 1.1 hi]",
            coarse_levels_setup_s=round(t_setup, 2))
    ctx.set_multigrid(None)
    for c in ctxs[1:]:
        c.close()
    return out


def time_call(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def consistent_suite(ctx, torch, k, reps=10):
    """The operator with consistent integration (2k+1 Gauss points): time per
    application, algorithmic bytes (7 nq^3 + 21 nq^2 numbers per cell, plus x
    and y), and its difference to the fast operator on a smooth field (the
    aliasing of the (k+1)-point rule)."""
    import synth_inputs as si
    xyz = ctx.dof_coordinates()
    fa, fb = si.terrain_coefficients()
    a, b = field_on_device(fa, xyz, torch), field_on_device(fb, xyz, torch)
    t0 = time.time()
    ctx.set_consistent(a, b)
    torch.cuda.synchronize()
    t_set = time.time() - t0
    x = field_on_device(si.rhs_terrain(0), xyz, torch)
    del xyz, a, b
    y = torch.empty_like(x)
    ms = time_call(lambda: ctx.apply_consistent(x, y), reps, torch)
    n = ctx.n_dofs
    nq, nd = 2 * k + 1, (k + 1) ** 3
    bpd = (7 * nq ** 3 + 21 * nq ** 2) * 8 / nd + 16
    yf = ctx.apply_operator(x)
    alias = float(torch.linalg.norm(yf - y) / torch.linalg.norm(y))
    # the same for a rough field (seeded normal entries)
    g = torch.Generator(device=x.device)
    g.manual_seed(7)
    xr = torch.randn(n, dtype=torch.float64, device=x.device, generator=g)
    ctx.apply_consistent(xr, y)
    yf = ctx.apply_operator(xr)
    alias_r = float(torch.linalg.norm(yf - y) / torch.linalg.norm(y))
    del xr
    out = dict(nq=nq, ms=round(ms, 3), gdofs=round(n / (ms * 1e-3) / 1e9, 3),
               alg_bytes_per_dof=round(bpd, 1), alg_GBs=round(bpd * n / (ms * 1e-3) / 1e9, 1),
               frac=round(bpd * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               set_consistent_s=round(t_set, 2), rel_diff_fast_vs_consistent_smooth=alias,
               rel_diff_fast_vs_consistent_random=alias_r)
    log(f"consistent integration: {out}")
    del x, y, yf
    return out


def consistent_mass_suite(hx, ctx, b, torch, reps=10):
    """The alpha-weighted mass with consistent integration (2k+1 points,
    beta = 0) solved by CG with the fast (k+1)-point mass-block inverse as
    preconditioner, against that fast inverse alone: the paper's two
    treatments of its modified mass matrix (an iterative solve with
    over-integration, or the direct tensor-product inverse with aliasing).
    Replaces the consistent data of the context."""
    import synth_inputs as si
    xyz = ctx.dof_coordinates()
    fa, _ = si.terrain_coefficients()
    a = field_on_device(fa, xyz, torch)
    del xyz
    ctx.set_consistent(a, torch.zeros_like(a))
    del a
    res = solve_suite(hx, ctx, b, torch, [
        ("consistent_mass_cg_fast_inverse", hx.default_params(
            method=0, rtol=1e-8, system=2, pc=hx.HX_PC_MASS_BLOCK))], "C3")
    z = torch.empty_like(b)
    ms_fast = time_call(lambda: ctx.apply_preconditioner(b, z, kind=hx.HX_PC_MASS_BLOCK), reps,
                        torch)
    x, _ = ctx.solve(b, params=hx.default_params(method=0, rtol=1e-12, system=2,
                                                 pc=hx.HX_PC_MASS_BLOCK))
    res["fast_inverse_ms"] = round(ms_fast, 3)
    res["rel_diff_fast_inverse_vs_consistent"] = float(torch.linalg.norm(z - x) /
                                                       torch.linalg.norm(x))
    log(f"C3 consistent mass: {res}")
    del x, z
    return res


def pressure_suite(hx, ctx, torch, label, forms, reps=10, fixed_point=False):
    """The pressure system of the IMEX stage (S = D - C A^-1 B) on the
    isothermal background: timing of S and its parts, FGMRES solves of
    S p = G - C A^-1 F, and (optionally) the fixed point from a state p*
    built, with the library itself, to be its solution."""
    import synth_inputs as si
    gamma, T = 1.4, si.TERRAIN
    xyz = ctx.dof_coordinates()
    frho, fh = si.terrain_pressure_fields(gamma)
    rho, h = field_on_device(frho, xyz, torch), field_on_device(fh, xyz, torch)
    ctx.set_pressure_system(rho, h, gamma, T["dt"])
    n = ctx.n_dofs
    p = field_on_device(si.rhs_terrain(5), xyz, torch)
    u3 = torch.stack([field_on_device(si.rhs_terrain(s), xyz, torch) for s in (6, 7, 8)])
    out = {}
    for name, part, arg in (("S", hx.HX_PS_SYSTEM, p), ("B", hx.HX_PS_GRAD, p),
                            ("C", hx.HX_PS_DIV, u3), ("A_inv_3", hx.HX_PS_VMASS_INV, u3),
                            ("D", hx.HX_PS_DMASS, p)):
        out[f"ms_{name}"] = round(time_call(lambda: ctx.apply_pressure_part(part, arg), reps, torch), 3)
    # algorithmic bytes per dof of the two face-coupled kernels (FP64)
    for name, bpd in (("B", 132.8), ("C", 142.4)):
        out[f"{name}_alg_GBs"] = round(bpd * n / (out[f"ms_{name}"] * 1e-3) / 1e9, 1)
    G = field_on_device(si.rhs_terrain(9), xyz, torch)
    b = ctx.pressure_rhs(u3, G)
    res = {}
    for name, prm in forms:
        x = torch.zeros_like(b)
        torch.cuda.synchronize()
        t0 = time.time()
        x, info = ctx.solve(b, x, prm)
        torch.cuda.synchronize()
        res[name] = dict(ms=round((time.time() - t0) * 1e3, 3), iters=info["iters"],
                         inner_iters=info["inner_iters"], true_rel_res=info["true_rel_res"],
                         status=hx.STATUS_NAMES[info["status"]])
        log(f"{label} pressure {name}: {res[name]}")
    out["solve"] = res
    if fixed_point:
        # p* = perturbed hydrostatic pressure; G chosen so that p* is the fixed point
        z = xyz[2]
        p_bg = 1e5 * torch.exp(-z / T["H"])
        p_star = p_bg * (1.0 + 0.02 * torch.sin(2 * np.pi * xyz[0] / T["Lx"])
                         * torch.cos(np.pi * z / T["Lz"]))
        h_star = gamma * p_star / ((gamma - 1.0) * rho)
        ctx.set_pressure_system(rho, h_star, gamma, T["dt"])
        F = 10.0 * rho * u3
        G = ctx.apply_pressure_part(hx.HX_PS_SYSTEM, p_star) + (G - ctx.pressure_rhs(F, G))
        pf = p_bg.clone()
        prm = hx.default_params(method=1, restart=30, rtol=1e-10, max_iter=5000,
                                pc=hx.HX_PC_BLOCK_JACOBI)
        torch.cuda.synchronize()
        t0 = time.time()
        pf, info = ctx.solve_pressure_fixed_point(rho, F, G, pf, gamma, T["dt"], params=prm,
                                                  max_fp_iters=30, fp_tol=1e-9)
        torch.cuda.synchronize()
        err = float(torch.linalg.norm(pf - p_star) / torch.linalg.norm(p_star))
        out["fixed_point"] = dict(ms=round((time.time() - t0) * 1e3, 1), fp_iters=info["fp_iters"],
                                  last_change=info["fp_change"], rel_error_vs_p_star=err,
                                  status=hx.STATUS_NAMES[info["status"]])
        log(f"{label} pressure fixed point: {out['fixed_point']}")
    del xyz, rho, h, p, u3, G, b
    return out


def kernels_suite(hx, ctx, torch, dev, dims, k, reps):
    """Every hot kernel of the path launched ``reps`` times on the timed mesh
    (for kernel traces and counters), with its mean time per launch from HIP
    events on the context's stream and its algorithmic bytes per dof:
    FP64 and FP32 operator, block Jacobi in both precisions, the learned
    correction (seeded random network), the consistent-integration operator,
    the multigrid restriction and prolongation to the 2x coarser channel, and
    the pressure parts B (gradient) and C (divergence)."""
    import synth_inputs as si
    n = ctx.n_dofs
    nd = (k + 1) ** 3
    xyz = ctx.dof_coordinates()
    x = field_on_device(si.rhs_terrain(0), xyz, torch)
    y = torch.empty_like(x)
    out = {}
    # a plain copy of known size (8 n bytes read, 8 n written): the scale of
    # the HBM byte counters
    y.copy_(x)
    torch.cuda.synchronize()
    log(f"copy calibration: {8 * n} bytes read, {8 * n} bytes written")

    def rec(name, fn, bpd, flops_per_dof=None):
        ms = time_call(fn, reps, torch)
        d = dict(ms=round(ms, 4), alg_bytes_per_dof=round(bpd, 2),
                 alg_GBs=round(bpd * n / (ms * 1e-3) / 1e9, 1))
        d["frac"] = round(d["alg_GBs"] / HBM_PEAK_GBS, 4)
        if flops_per_dof:
            d["TFLOPs"] = round(flops_per_dof * n / (ms * 1e-3) / 1e12, 2)
        out[name] = d
        log(f"kernels {name}: {d}")

    _, b64 = ctx.operator_info(hx.HX_F64)
    _, b32 = ctx.operator_info(hx.HX_F32)
    rec("operator_f64", lambda: ctx.apply_operator(x, y), b64 / n)
    x32, y32 = x.float(), torch.empty(n, dtype=torch.float32, device=dev)
    rec("operator_f32", lambda: ctx.apply_operator(x32, y32), b32 / n)
    nf = (k + 1) ** 2
    bj = (3 * nf + 3 * (k + 1) + 4) / nd       # S, l, c per cell, per dof
    rec("block_jacobi_f64", lambda: ctx.apply_preconditioner(x, y), 16 + 8 * bj)
    rec("block_jacobi_f32", lambda: ctx.apply_preconditioner(x32, y32), 8 + 4 * bj)
    del x32, y32
    # learned: block Jacobi, then the fused correction (reads r_K and the six
    # neighbour face layers, reads and writes z)
    n_in = nd + 6 * nf + 1
    ctx.set_network(si.mlp_init(5, n_in=n_in, n_out=nd))
    mlp_flops = 2 * (n_in * 256 + 256 * 256 + 256 * nd) / nd
    rec("learned_pc", lambda: ctx.apply_preconditioner(x, y, kind=hx.HX_PC_LEARNED),
        16 + 8 * bj + 8 * (nd + 6 * nf) / nd + 16, mlp_flops)
    # consistent integration
    fa, fb = si.terrain_coefficients()
    ctx.set_consistent(field_on_device(fa, xyz, torch), field_on_device(fb, xyz, torch))
    nq = 2 * k + 1
    rec("operator_consistent", lambda: ctx.apply_consistent(x, y),
        (7 * nq ** 3 + 21 * nq ** 2) * 8 / nd + 16)
    # multigrid transfers to the 2x coarser channel
    nx, ny, nz = dims
    mc = si.terrain_mesh(nx // 2, ny // 2, nz // 2, g=4)
    cc, xc, _ = setup(hx.HelmDG, mc, k, torch, dev)
    del mc, xc
    ctx.set_multigrid(cc, *si.refinement_parents(nx // 2, ny // 2, nz // 2))
    yc = torch.empty(cc.n_dofs, dtype=torch.float64, device=dev)
    rec("mg_restrict", lambda: ctx.mg_transfer(0, x, yc), 8 + 8 / 8)
    rec("mg_prolong", lambda: ctx.mg_transfer(1, yc, y), 16 + 8 / 8)
    ctx.set_multigrid(None)
    cc.close()
    del yc
    # pressure parts
    gamma, T = 1.4, si.TERRAIN
    frho, fh = si.terrain_pressure_fields(gamma)
    ctx.set_pressure_system(field_on_device(frho, xyz, torch), field_on_device(fh, xyz, torch),
                            gamma, T["dt"])
    u3 = torch.stack([field_on_device(si.rhs_terrain(s_), xyz, torch) for s_ in (6, 7, 8)])
    rec("pressure_B", lambda: ctx.apply_pressure_part(hx.HX_PS_GRAD, x), 132.8)
    rec("pressure_C", lambda: ctx.apply_pressure_part(hx.HX_PS_DIV, u3), 142.4)
    del u3, xyz, x, y
    return out


def _omp_threads(n=None):
    """Set (n given) or read the OpenMP thread count of the calling thread,
    which runs the oracle's parallel regions."""
    import ctypes
    try:
        gomp = ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None
    if n is not None:
        gomp.omp_set_num_threads(int(n))
    return int(gomp.omp_get_max_threads())


def _cpu_model():
    """The host CPU model as lscpu reports it (else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _terrain_sample(nx, ny, layers):
    """The first nx x ny columns and bottom `layers` cell layers of the
    256x64x64 terrain channel (same cell sizes, map and fields)."""
    import synth_inputs as si
    T = si.TERRAIN
    hx_, hy, hz = T["Lx"] / 256, T["Ly"] / 64, T["Lz"] / 64
    return si.box_mesh(nx, ny, layers, lo=(-T["Lx"] / 2, 0.0, 0.0),
                       hi=(-T["Lx"] / 2 + nx * hx_, ny * hy, layers * hz),
                       periodic=(nx == 256, ny == 64, False), g=4, mapping=si.terrain_mapping)


def cpu_baseline(layers: int, solutions):
    """The FP64 oracle on the host cores (a baseline, not a target), and the
    error of each kept GPU solution against the oracle's solution.

    * value: oracle matvec GDoF/s on the bottom `layers` cell layers of the
      256x64x64 channel, all cores; the same on a 1,024-cell sample with one
      thread;
    * the periodic unit cube (4^3, Q2) and the 32x8x16 channel: oracle
      matvec, and CG with the separable block to 1e-10 (cube, run to the end)
      and to 1e-8 (channel: time per iteration measured over 3 iterations,
      times the 72 iterations the oracle's own solve takes, from the stored
      reference solve);
    * err_vs_oracle per kept solution: ||x - x*|| / ||x*|| against a dense
      solve (cube Q2), the oracle's CG to 1e-13 (cube Q4) or the stored
      oracle solution of the 32x8x16 channel (1e-13)."""
    import oracle
    import synth_inputs as si
    threads = _omp_threads()
    rec = dict(unit="GDoF/s", kind="oracle", cpu_model=_cpu_model(),
               nproc=len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count())
    # all-core matvec on the large sample
    m = _terrain_sample(256, 64, layers)
    p = oracle.Problem(m, 4)
    p.set_coefficient_functions(*si.terrain_coefficients())
    x = si.rhs_terrain(0)(*p.dof_coords())
    t0 = time.time()
    p.apply(x)
    dt = time.time() - t0
    rec.update(value=p.n_dofs / dt / 1e9, cores=threads,
               sample=f"FP64 oracle matvec on the bottom {layers} cell layers of the 256x64x64 "
                      f"Q4 terrain channel ({m.n_cells} cells, {p.n_dofs} dofs), {dt:.2f} s")
    # one thread, 1,024 cells of the same channel
    m1 = _terrain_sample(256, 4, 1)
    p1 = oracle.Problem(m1, 4)
    p1.set_coefficient_functions(*si.terrain_coefficients())
    x1 = si.rhs_terrain(0)(*p1.dof_coords())
    _omp_threads(1)
    t0 = time.time()
    p1.apply(x1)
    dt1 = time.time() - t0
    used1 = _omp_threads()
    _omp_threads(threads)
    rec["one_thread"] = dict(value=p1.n_dofs / dt1 / 1e9, cores=used1,
                             sample=f"oracle matvec, {m1.n_cells} cells of the same channel, {dt1:.2f} s")
    # the periodic unit cube, Q2: matvec and CG to 1e-10
    errs = {}
    pc = oracle.Problem(si.cube_mesh(4), 2)
    pc.set_coefficient_functions(*si.const_coefficients(1.0, 0.01))
    bc = si.rhs_cube(0)(*pc.dof_coords())
    t0 = time.time()
    pc.apply(bc)
    t_mv = time.time() - t0
    t0 = time.time()
    xc, ic = oracle.solvers.cg(pc.apply, bc, precond=pc.bj_apply, rtol=1e-10)
    t_cg = time.time() - t0
    rec["cube4_q2"] = {"matvec_ms": round(t_mv * 1e3, 2), "cg_bj_1e-10_ms": round(t_cg * 1e3, 1),
                        "cg_iters": ic.iters}
    xd = np.linalg.solve(pc.assemble_dense(), bc)
    for name, xg in solutions.get("cube4_q2", {}).items():
        errs.setdefault("cube4_q2", {})[name] = float(np.linalg.norm(xg - xd) / np.linalg.norm(xd))
    # the periodic unit cube, Q4 (the learned form's mesh)
    p5 = oracle.Problem(si.cube_mesh(4), 4)
    p5.set_coefficient_functions(*si.const_coefficients(1.0, 0.01))
    b5 = si.rhs_cube(101)(*p5.dof_coords())
    x5, i5 = oracle.solvers.cg(p5.apply, b5, precond=p5.bj_apply, rtol=1e-13)
    for name, xg in solutions.get("cube4_q4", {}).items():
        errs.setdefault("cube4_q4", {})[name] = float(np.linalg.norm(xg - x5) / np.linalg.norm(x5))
    # the 32x8x16 channel: matvec, CG per iteration, stored 1e-13 solution
    p2 = oracle.Problem(si.terrain_mesh(32, 8, 16, g=4), 4)
    p2.set_coefficient_functions(*si.terrain_coefficients())
    b2 = si.rhs_terrain(0)(*p2.dof_coords())
    t0 = time.time()
    p2.apply(b2)
    t_mv2 = time.time() - t0
    t0 = time.time()
    oracle.solvers.cg(p2.apply, b2, precond=p2.bj_apply, rtol=1e-30, max_iter=3)
    t_it = (time.time() - t0) / 3.0
    ref = os.path.join(ROOT, "tests", "golden", "terrain32x8x16_k4_rhs0_solution")
    meta = {}
    for line in open(ref + ".txt"):
        if not line.startswith("#"):
            kk, vv = line.split()
            meta[kk] = float(vv)
    rec["terrain32x8x16"] = {"matvec_ms": round(t_mv2 * 1e3, 1),
                             "cg_bj_ms_per_iter": round(t_it * 1e3, 1),
                             "cg_bj_1e-8_ms_projected": round(t_it * 1e3 * meta["iterations_to_1e-8"], 0),
                             "oracle_iters_to_1e-8": int(meta["iterations_to_1e-8"])}
    xs = np.load(ref + ".npy")
    for name, xg in solutions.get("terrain32x8x16", {}).items():
        errs.setdefault("terrain32x8x16", {})[name] = float(np.linalg.norm(xg - xs) / np.linalg.norm(xs))
    return rec, errs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=64)
    ap.add_argument("--nz", type=int, default=64)
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--solves", choices=["all", "large", "multigrid"], default="all",
                    help="'large': only the solves on the timed mesh; 'multigrid': only CG "
                         "with the multigrid V-cycle on it (both for profiling)")
    ap.add_argument("--degree", type=int, default=4,
                    help="polynomial degree (default 4, the benchmark's)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-layers", type=int, default=4)
    ap.add_argument("--no-fp32", action="store_true", help="skip the timing of the FP32 operator")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the timed applications (no extra timing windows), for profilers")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="also run a plain device copy of the x vector (for counter scaling)")
    ap.add_argument("--kernels", action="store_true",
                    help="only launch every hot kernel --steps times on the mesh and report "
                         "each one's time and algorithmic bandwidth (for profilers)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library does "
              "not shard the mesh across GPUs.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2505_00384_amd as hx
    import synth_inputs as si

    dev = torch.device("cuda:0")
    k = args.degree
    log(f"building mesh {args.nx}x{args.ny}x{args.nz}")
    mesh = si.terrain_mesh(args.nx, args.ny, args.nz, g=4)
    setup_times = {}
    ctx, xyz, t_setup = setup(hx.HelmDG, mesh, k, torch, dev, setup_times)
    n = ctx.n_dofs
    log(f"setup {t_setup:.2f} s, {n} dofs")
    del mesh
    if args.kernels:
        res = kernels_suite(hx, ctx, torch, dev, (args.nx, args.ny, args.nz), k, args.steps)
        ctx.close()
        print(json.dumps({"kernels": res, "config": {"mesh": f"{args.nx}x{args.ny}x{args.nz}",
                                                     "degree": k, "n_dofs": n}}), flush=True)
        return
    x = rhs_on_device(xyz, 0, torch)
    del xyz
    y = torch.empty_like(x)
    ms = time_matvec(ctx, x, y, args.steps, args.warmup, torch)
    gdofs = n / (ms * 1e-3) / 1e9
    counts, op_bytes = ctx.operator_info(hx.HX_F64)
    achieved = op_bytes / (ms * 1e-3) / 1e9
    log(f"FP64 matvec {ms:.4f} ms, {gdofs:.2f} GDoF/s, {achieved:.0f} GB/s algorithmic "
        f"({op_bytes / n:.1f} B/dof; {counts})")
    extra = {}
    if not args.profile_run:
        extra["operator"] = operator_windows(hx, ctx, x, y, torch, n, op_bytes, counts)
        log(f"operator: {extra['operator']}")
    if not args.no_fp32:
        x32 = x.float()
        y32 = torch.empty_like(x32)
        ms32 = time_matvec(ctx, x32, y32, args.steps, args.warmup, torch)
        _, b32 = ctx.operator_info(hx.HX_F32)
        extra["fp32_matvec"] = dict(ms=round(ms32, 4), gdofs=round(n / (ms32 * 1e-3) / 1e9, 3),
                                    alg_GBs=round(b32 / (ms32 * 1e-3) / 1e9, 1),
                                    frac=round(b32 / (ms32 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
        log(f"FP32 matvec {ms32:.4f} ms")
        del x32, y32
    if args.copy_calibrate:
        # a plain copy of known size: reads and writes 8 n bytes each
        y.copy_(x)
        torch.cuda.synchronize()
        log(f"copy calibration: {8 * n} bytes read, {8 * n} bytes written")
    traffic = read_traffic(n) if (k == 4 and (args.nx, args.ny, args.nz) == (256, 64, 64)) else None
    roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(achieved / HBM_PEAK_GBS, 4), traffic=traffic)

    solve = {}
    kept = {}      # GPU solutions kept for the oracle comparison
    pressure = {}
    consistent = None
    if not args.no_solve:
        b = x
        forms = [
            ("fp64_fgmres_bj", hx.default_params(method=1, restart=30, rtol=1e-8, pc=hx.HX_PC_BLOCK_JACOBI)),
            ("mixed_fp32_inner", hx.default_params(method=1, restart=10, rtol=1e-8, mixed=1, inner_iters=32)),
            # the minimal mixed form: FP32 operator and block Jacobi inside FP64 FGMRES
            ("mixed_fp32_minimal", hx.default_params(method=1, restart=30, rtol=1e-8, mixed=2)),
        ]
        # SPD operator: CG with block Jacobi and with the paper's Helmholtz
        # (volume-diagonal) preconditioner
        cg_forms = [
            ("fp64_cg_bj", hx.default_params(method=0, rtol=1e-8, pc=hx.HX_PC_BLOCK_JACOBI)),
            ("fp64_cg_helmholtz_diag", hx.default_params(method=0, rtol=1e-8, max_iter=20000,
                                                         pc=hx.HX_PC_HELMHOLTZ_DIAG)),
        ]
        del y
        # learned form: network trained on the periodic unit cube at the same
        # degree with the library's own kernels, then used on every mesh
        w_net, t_train, learned_form = None, None, []
        if args.solves == "all":
            from paper_2505_00384_amd import learned
            t0 = time.time()
            F, T = learned.generate_pairs(100000, seed=0, k=k, log=log)
            ctx.set_network(learned.init_weights(ctx, seed=0))
            learned.train(ctx, F, T, steps=3000, batch=2048, lr=1e-3, log=log, log_every=1000)
            t_train = time.time() - t0
            del F, T
            w_net = ctx.get_network()
            learned_form = [("learned_fgmres", hx.default_params(method=1, restart=30, rtol=1e-8,
                                                                 pc=hx.HX_PC_LEARNED))]
        solve[f"terrain{args.nx}x{args.ny}x{args.nz}"] = solve_suite(
            hx, ctx, b, torch, [] if args.solves == "multigrid" else forms + cg_forms + learned_form,
            "C3")
        # CG with the Chebyshev polynomial (degree 4) around block Jacobi, its
        # interval from 20 Lanczos steps on a random vector (timed apart)
        gen = torch.Generator(device=dev)
        gen.manual_seed(3)
        rv = torch.randn(n, dtype=torch.float64, device=dev, generator=gen)
        torch.cuda.synchronize()
        t0 = time.time()
        lo, hi = ctx.estimate_eigenvalues(rv, 20)
        torch.cuda.synchronize()
        t_est = (time.time() - t0) * 1e3
        del rv
        if args.solves != "multigrid":
            ctx.set_chebyshev(4, lo, 1.1 * hi)
            cheb = solve_suite(hx, ctx, b, torch, [
                ("fp64_cg_chebyshev4_bj", hx.default_params(method=0, rtol=1e-8,
                                                            pc=hx.HX_PC_CHEBYSHEV))], "C3")
            cheb["fp64_cg_chebyshev4_bj"].update(lanczos_ms=round(t_est, 1), lanczos_lo=lo,
                                                 lanczos_hi=hi)
            solve[f"terrain{args.nx}x{args.ny}x{args.nz}"].update(cheb)
        if args.solves != "multigrid":
            consistent = consistent_suite(ctx, torch, k)
        solve[f"terrain{args.nx}x{args.ny}x{args.nz}"].update(
            multigrid_suite(hx, ctx, b, torch, dev, (args.nx, args.ny, args.nz), k, (lo, hi),
                            consistent=consistent is not None))
        if args.solves != "multigrid":
            consistent["weighted_mass"] = consistent_mass_suite(hx, ctx, b, torch)
            # the pressure system of the stage on the same mesh: FGMRES with
            # the block Jacobi of the Helmholtz-type operator
            pressure[f"terrain{args.nx}x{args.ny}x{args.nz}"] = pressure_suite(
                hx, ctx, torch, "C3",
                [("fgmres_bj", hx.default_params(method=1, system=1, restart=30, rtol=1e-8,
                                                 max_iter=5000, pc=hx.HX_PC_BLOCK_JACOBI))])
        ctx.close()
    if not args.no_solve and args.solves == "all":
        del b, x
        torch.cuda.empty_cache()
        m2 = si.terrain_mesh(32, 8, 16, g=4)
        ctx2, xyz2, _ = setup(hx.HelmDG, m2, k, torch, dev)
        b2 = rhs_on_device(xyz2, 0, torch)
        forms2 = forms + cg_forms + [
            ("fp64_cg_mass_diag", hx.default_params(method=0, rtol=1e-8, max_iter=20000,
                                                    pc=hx.HX_PC_MASS_DIAG)),
            ("fp64_fgmres_helmholtz_diag", hx.default_params(method=1, restart=30, rtol=1e-8,
                                                             max_iter=20000,
                                                             pc=hx.HX_PC_HELMHOLTZ_DIAG))]
        # the learned form with the network trained above
        ctx2.set_network(w_net)
        forms2 += learned_form
        solve["terrain32x8x16"] = solve_suite(hx, ctx2, b2, torch, forms2, "C2",
                                              keep=kept.setdefault("terrain32x8x16", {}))
        solve["learned_training_s"] = round(t_train, 2)
        w = w_net
        solve["terrain32x8x16_refined"] = nonconforming_suite(hx, torch, dev, k)
        log(f"nonconforming: {solve['terrain32x8x16_refined']}")
        pressure["terrain32x8x16"] = pressure_suite(hx, ctx2, torch, "C2", [
            ("fgmres_helmholtz_diag", hx.default_params(method=1, system=1, restart=30, rtol=1e-8,
                                                        max_iter=20000, pc=hx.HX_PC_HELMHOLTZ_DIAG)),
            ("fgmres_mass_diag", hx.default_params(method=1, system=1, restart=30, rtol=1e-8,
                                                   max_iter=20000, pc=hx.HX_PC_MASS_DIAG)),
            ("fgmres_bj", hx.default_params(method=1, system=1, restart=30, rtol=1e-8,
                                            max_iter=20000, pc=hx.HX_PC_BLOCK_JACOBI)),
            ("fgmres_inner_cg", hx.default_params(method=1, system=1, restart=10, rtol=1e-8,
                                                  mixed=1, inner_iters=32))], fixed_point=True)
        ctx2.close()
        # the periodic unit cube: degree 2 CG + block Jacobi to 1e-10, and the
        # learned form at degree 4 on the same mesh
        m1 = si.cube_mesh(4)
        c1 = hx.HelmDG(0)
        c1.setup_mesh(2, m1.nodes, m1.nbr, 1)
        x1 = c1.dof_coordinates()
        ones = torch.ones(c1.n_dofs, dtype=torch.float64, device=dev)
        c1.set_coefficients(ones, 0.01 * ones, 2.0)
        b1 = field_on_device(si.rhs_cube(0), x1, torch)
        solve["cube4_q2"] = solve_suite(hx, c1, b1, torch, [
            ("fp64_cg_bj_1e-10", hx.default_params(method=0, rtol=1e-10))], "C1",
            keep=kept.setdefault("cube4_q2", {}))
        c1.close()
        c5 = hx.HelmDG(0)
        c5.setup_mesh(4, m1.nodes, m1.nbr, 1)
        x5 = c5.dof_coordinates()
        ones = torch.ones(c5.n_dofs, dtype=torch.float64, device=dev)
        c5.set_coefficients(ones, 0.01 * ones, 2.0)
        c5.set_network(w)
        b5 = field_on_device(si.rhs_cube(101), x5, torch)
        solve["cube4_q4"] = solve_suite(hx, c5, b5, torch, [
            ("fp64_fgmres_bj", hx.default_params(method=1, restart=30, rtol=1e-8)),
            ("learned_fgmres", hx.default_params(method=1, restart=30, rtol=1e-8, pc=hx.HX_PC_LEARNED))],
            "C5", keep=kept.setdefault("cube4_q4", {}))
        c5.close()
    else:
        ctx.close()

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cpu, errs = cpu_baseline(args.cpu_layers, kept)
        for wl, d in errs.items():
            for name, e in d.items():
                solve[wl][name]["err_vs_oracle"] = e
        log(f"cpu baseline {cpu}")

    rec = {
        "metric": "Helmholtz matvec GDoF/s (% HBM peak); time-to-1e-8 solve: FP64 vs mixed/learned",
        "value": round(gdofs, 3), "unit": "GDoF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"terrain-following channel {args.nx}x{args.ny}x{args.nz} cells, DG Q{k}, "
                               "isothermal background coefficients, SIP penalty 2",
                   "n_dofs": n, "degree": k, "geometry_degree": 4},
        "roofline": roof,
        "cpu_baseline": cpu,
        "solve": solve,
        "pressure_system": pressure,
        "consistent_integration": consistent,
        "setup": setup_times,
        **extra,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
