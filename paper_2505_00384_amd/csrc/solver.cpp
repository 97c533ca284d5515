// Host drivers of the Krylov solves (the paper's pressure solve: PCG for
// symmetric positive-definite systems, GMRES with a Jacobi-type
// preconditioner, section 3.1).  All vector work runs in HIP kernels on the
// context stream; the host only takes the scalar decisions.
//
//  * CG: preconditioned conjugate gradients in FP64.
//  * FGMRES(m): right-preconditioned flexible GMRES with classical
//    Gram-Schmidt applied twice (CGS2), either as two block-dot/update pairs
//    per step or with the second pass delayed and fused into the next step
//    (two passes over the basis per step instead of four), Givens rotations
//    on the host, explicit residual b - A x at every restart.
//  * Mixed precision: the FGMRES preconditioner is an inner FP32 PCG with
//    FP32 operator and FP32 block Jacobi, run for a fixed number of
//    iterations with all scalars kept on the device; the outer residual,
//    orthogonalisation and update stay FP64 (iterative refinement through the
//    explicit FP64 residual at each restart).
//  * Learned: block Jacobi plus the network correction; if the residual
//    estimate stalls over stall_window iterations, or the preconditioned
//    vector is not finite (its Hessenberg column is then not finite and the
//    Givens step rejects it), the solver restarts from the current x with
//    block Jacobi.
#include <chrono>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace hx {
namespace {

constexpr int64_t SC_OFF = 1024 * 66;   // device scalar area inside c->red

struct Timer {
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    double op = 0, pc = 0, orth = 0;
    bool ok = false;
    explicit Timer(bool on)
    {
        if (!on) return;
        ok = true;
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) ok = false;
    }
    ~Timer()
    {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
    void rec(int i, hipStream_t s)
    {
        if (ok) (void)hipEventRecord(ev[i], s);
    }
    float span(int i, int j)
    {
        float t = 0;
        return hipEventElapsedTime(&t, ev[i], ev[j]) == hipSuccess ? t : 0.0f;
    }
    // after a stream sync (FGMRES order ev0 < ev1 < ev2 < ev3):
    // pc = ev0..1, op = ev1..2, orth = ev2..3
    void acc()
    {
        if (!ok) return;
        pc += span(0, 1);
        op += span(1, 2);
        orth += span(2, 3);
    }
    // CG order ev1 < ev2 < ev0 < ev3: op = ev1..2, p.q = ev2..0, fused
    // updates and preconditioner = ev0..3
    void acc_cg()
    {
        if (!ok) return;
        op += span(1, 2);
        orth += span(2, 0);
        pc += span(0, 3);
    }
};

hx_status ensure_work(hx_ctx *c, size_t n64, size_t n32)
{
    if (n64 > c->work64_len) {
        dfree((void **)&c->work64);
        c->work64_len = 0;
        hx_status s = dalloc(c, (void **)&c->work64, sizeof(double) * n64);
        if (s != HX_OK) return s;
        c->work64_len = n64;
    }
    if (n32 > c->work32_len) {
        dfree((void **)&c->work32);
        c->work32_len = 0;
        hx_status s = dalloc(c, (void **)&c->work32, sizeof(float) * n32);
        if (s != HX_OK) return s;
        c->work32_len = n32;
    }
    return HX_OK;
}

// inner FP32 PCG for `iters` iterations on A32 z = v (FP64 in/out) with the
// FP32 form of preconditioner pc (block Jacobi, the cell mass blocks, a
// diagonal kind or none);
// scalars on the device, each step fused around the preconditioner (one pass
// over x, r, p, q and z).  w32: 5 float vectors.
hx_status inner_fp32(hx_ctx *c, int pc, const double *v, double *z, float *w32, int iters,
                     int *count)
{
    const int64_t n = c->n_dofs;
    float *x = w32, *r = w32 + n, *zz = w32 + 2 * n, *p = w32 + 3 * n, *q = w32 + 4 * n;
    double *sc = c->red + SC_OFF + 512;   // [0] rz, [1] pq, [2] rz_new, [3] rr
    HX_HIP(c, blas_cast64to32(c, n, v, r, nullptr));
    HX_HIP(c, blas_fill32(c, n, 0.0f, x));
    switch (pc) {
    case HX_PC_BLOCK_JACOBI: HX_HIP(c, launch_bj32(c, r, zz)); break;
    case HX_PC_HELMHOLTZ_DIAG: HX_HIP(c, launch_diag32(c, 0, r, zz)); break;
    case HX_PC_MASS_DIAG: HX_HIP(c, launch_diag32(c, 1, r, zz)); break;
    case HX_PC_MASS_BLOCK: HX_HIP(c, launch_massinv32(c, r, zz)); break;
    default:
        HX_HIP(c, hipMemcpyAsync(zz, r, sizeof(float) * n, hipMemcpyDeviceToDevice, c->stream));
    }
    HX_HIP(c, hipMemcpyAsync(p, zz, sizeof(float) * n, hipMemcpyDeviceToDevice, c->stream));
    HX_HIP(c, blas_dot32(c, n, r, zz, sc + 0));
    CgLoop lp;   // the current r.z in sc[lp.cur]
    for (int it = 0; it < iters; ++it) {
        // p.q: partial sums left for the step kernel, or summed into sc[1]
        int npq = 0;
        HX_HIP(c, launch_apply32_dot(c, p, q, sc + 1, &npq));
        if (it + 1 == iters) {
            HX_HIP(c, cg32_step_x(c, n, x, r, p, q, sc + lp.cur, npq > 0 ? c->pqpart : nullptr, npq));
            break;
        }
        int fl = 0;
        HX_HIP(c, cg_step_pc32(c, pc, x, r, p, q, zz, sc, &fl, npq, &lp));
        HX_HIP(c, cg_step_p32(c, zz, p, sc, fl, &lp));
    }
    HX_HIP(c, blas_cast32to64(c, n, x, z, nullptr));
    *count += iters;
    return HX_OK;
}

// one FP32 application of preconditioner pc to the FP64 vector v (the
// minimal mixed form): z = (double) M32^-1 (float) v.  w32: 2 float vectors.
hx_status once_fp32(hx_ctx *c, int pc, const double *v, double *z, float *w32)
{
    const int64_t n = c->n_dofs;
    float *r = w32, *zz = w32 + n;
    HX_HIP(c, blas_cast64to32(c, n, v, r, nullptr));
    switch (pc) {
    case HX_PC_BLOCK_JACOBI: HX_HIP(c, launch_bj32(c, r, zz)); break;
    case HX_PC_HELMHOLTZ_DIAG: HX_HIP(c, launch_diag32(c, 0, r, zz)); break;
    case HX_PC_MASS_DIAG: HX_HIP(c, launch_diag32(c, 1, r, zz)); break;
    case HX_PC_MASS_BLOCK: HX_HIP(c, launch_massinv32(c, r, zz)); break;
    default: zz = r;
    }
    HX_HIP(c, blas_cast32to64(c, n, zz, z, nullptr));
    return HX_OK;
}

hx_status precondition(hx_ctx *c, int pc, int mixed, int inner_iters, const double *v, double *z,
                       float *w32, int *inner_count)
{
    if (mixed == 2) return once_fp32(c, pc, v, z, w32);
    if (mixed) return inner_fp32(c, pc, v, z, w32, inner_iters, inner_count);
    switch (pc) {
    case HX_PC_NONE: HX_HIP(c, blas_copy(c, c->n_dofs, v, z)); return HX_OK;
    case HX_PC_BLOCK_JACOBI: HX_HIP(c, launch_bj64(c, v, z)); return HX_OK;
    case HX_PC_LEARNED: return mlp_precondition(c, v, z);
    case HX_PC_HELMHOLTZ_DIAG: HX_HIP(c, launch_diag64(c, 0, v, z)); return HX_OK;
    case HX_PC_MASS_DIAG: HX_HIP(c, launch_diag64(c, 1, v, z)); return HX_OK;
    case HX_PC_MASS_BLOCK: HX_HIP(c, launch_massinv64(c, v, z)); return HX_OK;
    case HX_PC_CHEBYSHEV: HX_HIP(c, cheb_apply64(c, v, z)); return HX_OK;
    case HX_PC_MULTIGRID: HX_HIP(c, mg_vcycle64(c, v, z)); return HX_OK;
    case HX_PC_MULTIGRID_MIXED: HX_HIP(c, mg_vcycle_mixed(c, v, z)); return HX_OK;
    default: return fail(c, HX_ERR_ARG, "unknown preconditioner %d", pc);
    }
}

double now_ms()
{
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// the additions of the device's sum256, in its order: 256 thread sums of
// strided elements, each wave folded by halving distances, the four wave
// sums in order
double host_sum256(const double *p, int nb)
{
    double th[256];
    for (int t = 0; t < 256; ++t) {
        double s = 0.0;
        for (int i = t; i < nb; i += 256) s += p[i];
        th[t] = s;
    }
    double tot = 0.0;
    for (int wv = 0; wv < 4; ++wv) {
        double *v = th + 64 * wv;
        for (int o = 32; o > 0; o >>= 1)
            for (int i = 0; i < o; ++i) v[i] = v[i] + v[i + o];
        tot += v[0];
    }
    return tot;
}

namespace {

hx_status read_scalars(hx_ctx *c, const double *dev, int m, double *host)
{
    HX_HIP(c, hipMemcpyAsync(c->red_host, dev, sizeof(double) * m, hipMemcpyDeviceToHost, c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    std::memcpy(host, c->red_host, sizeof(double) * m);
    return HX_OK;
}

// ------------------------------------------------------------------- CG
// Preconditioned CG with its scalars on the device: per step one operator
// application that also sums p.q, one fused kernel (x and r updates,
// preconditioner, r.z and r.r) and the update of p.  The host reads |r|^2
// of step k while step k+1 runs, so the stream never waits for the host; the
// solve stops one step after the test first passes.
// y = M x or y = b - M x for the system being solved: the Helmholtz-type
// operator, the pressure system S = D - C A^-1 B, or the Helmholtz-type
// operator with consistent integration (2k+1 points)
hipError_t sys_apply(hx_ctx *c, const hx_solve_params *prm, const double *x, double *y,
                     const double *b);

// the operator of an Arnoldi step: FP64, or FP32 in the minimal mixed form
// (w32 + 2 n .. + 4 n: the FP32 copies of x and y)
hipError_t step_apply(hx_ctx *c, const hx_solve_params *prm, const double *x, double *y, float *w32)
{
    if (prm->mixed != 2) return sys_apply(c, prm, x, y, nullptr);
    const int64_t n = c->n_dofs;
    float *x32 = w32 + 2 * n, *y32 = w32 + 3 * n;
    hipError_t e = blas_cast64to32(c, n, x, x32, nullptr);
    if (e == hipSuccess) e = launch_apply32(c, x32, y32, nullptr);
    if (e == hipSuccess) e = blas_cast32to64(c, n, y32, y, nullptr);
    return e;
}

hipError_t sys_apply(hx_ctx *c, const hx_solve_params *prm, const double *x, double *y,
                     const double *b)
{
    if (prm->system == 1) return press_apply64(c, x, y, b);
    if (prm->system == 2) {
        hipError_t e = launch_apply_q(c, x, y);
        if (e == hipSuccess && b) e = blas_axpby(c, c->n_dofs, 1.0, b, -1.0, y);
        return e;
    }
    return launch_apply64(c, x, y, b);
}

// q = M p and dst = p.q (the operator kernel sums p.q itself for system 0
// and, when *npq > 0 on return, leaves its partial sums for the step kernel)
hipError_t sys_apply_dot(hx_ctx *c, const hx_solve_params *prm, const double *p, double *q,
                         double *dst, int *npq)
{
    *npq = 0;
    if (prm->system == 0) return launch_apply64_dot(c, p, q, dst, npq);
    hipError_t e = sys_apply(c, prm, p, q, nullptr);
    if (e == hipSuccess) e = blas_dot(c, c->n_dofs, p, q, dst);
    return e;
}

hx_status solve_cg(hx_ctx *c, const hx_solve_params *prm, const double *b, double *x,
                   hx_solve_info *info, Timer &tm)
{
    const int64_t n = c->n_dofs;
    hx_status s = ensure_work(c, 4 * (size_t)n, 0);
    if (s != HX_OK) return s;
    double *r = c->work64, *z = r + n, *p = z + n, *q = p + n;
    double *sc = c->red + SC_OFF;          // [0] rz, [1] pq, [2] rz_new, [3] rr, [4] bb
    double h[2];
    HX_HIP(c, blas_dot(c, n, b, b, sc + 4));
    if (prm->x0_mode == 1) {
        HX_HIP(c, sys_apply(c, prm, x, r, b));
    } else {
        HX_HIP(c, blas_fill(c, n, 0.0, x));
        HX_HIP(c, blas_copy(c, n, b, r));
    }
    HX_HIP(c, blas_dot(c, n, r, r, sc + 3));
    if ((s = read_scalars(c, sc + 3, 2, h)) != HX_OK) return s;
    const double nb = std::sqrt(h[1]);
    double rel = nb > 0 ? std::sqrt(h[0]) / nb : 0.0;
    if (nb == 0.0) {
        HX_HIP(c, blas_fill(c, n, 0.0, x));
        info->true_rel_res = 0.0;
        return HX_OK;
    }
    int dummy = 0;
    if ((s = precondition(c, prm->pc, 0, 0, r, z, nullptr, &dummy)) != HX_OK) return s;
    HX_HIP(c, blas_copy(c, n, z, p));
    HX_HIP(c, blas_dot(c, n, r, z, sc + 0));
    if (rel <= prm->rtol || prm->max_iter < 1) {
        info->iters = 0;
        info->history_len = 0;
        return HX_OK;
    }
    // two steps in flight: slot k % 2 of the pinned buffer, events and timers
    hipEvent_t done[2] = {nullptr, nullptr};
    for (auto &e : done)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return fail(c, HX_ERR_DEVICE, "hipEventCreate failed");
    Timer tb(true);
    Timer *tms[2] = {&tm, &tb};
    double *hr = c->pin_host;   // slots 0, 1 (device-mapped: the reduction may write them)
    auto cleanup = [&]() {
        for (auto &e : done)
            if (e) (void)hipEventDestroy(e);
    };
    int it = 0, checked = 0;
    bool stop = false;
    hx_status err = HX_OK;
    CgLoop lp;   // the current r.z in sc[lp.cur]
    // rel of step k, once its copy has landed
    auto check = [&](int k) -> bool {
        if (hipEventSynchronize(done[k % 2]) != hipSuccess) {
            err = fail(c, HX_ERR_DEVICE, "CG: event wait failed");
            return true;
        }
        tms[k % 2]->acc_cg();
        const double rk = std::sqrt(hr[k % 2]) / nb;
        if (info->history && k < info->history_len) info->history[k] = rk;
        checked = k + 1;
        return !(rk > prm->rtol) || !std::isfinite(rk);
    };
    while (it < prm->max_iter && !stop) {
        Timer &t = *tms[it % 2];
        t.rec(1, c->stream);
        int npq = 0;
        if (hipSuccess != sys_apply_dot(c, prm, p, q, sc + 1, &npq)) { err = fail(c, HX_ERR_DEVICE, "CG: apply"); break; }
        t.rec(2, c->stream);
        t.rec(0, c->stream);
        int fl = 0;
        if (hipSuccess != cg_step_pc64(c, prm->pc, x, r, p, q, z, sc, c->pin_dev + it % 2, &fl, npq, &lp)) { err = fail(c, HX_ERR_DEVICE, "CG: step"); break; }
        t.rec(3, c->stream);
        if (hipSuccess != cg_step_p64(c, z, p, sc, fl, &lp)) { err = fail(c, HX_ERR_DEVICE, "CG: p update"); break; }
        // |r|^2 for the host: written by the reduction itself, else copied
        if ((!(fl & CG_RR_ON_HOST) &&
             hipSuccess != hipMemcpyAsync(hr + it % 2, sc + 3, sizeof(double), hipMemcpyDeviceToHost,
                                          c->stream)) ||
            hipSuccess != hipEventRecord(done[it % 2], c->stream)) {
            err = fail(c, HX_ERR_DEVICE, "CG: copy");
            break;
        }
        ++it;
        // test the previous step while this one runs
        if (it >= 2 && check(it - 2)) stop = true;
    }
    // the steps still in flight
    while (err == HX_OK && checked < it) check(checked);
    cleanup();
    tm.op += tb.op;
    tm.pc += tb.pc;
    tm.orth += tb.orth;
    if (err != HX_OK) return err;
    info->iters = it;
    info->history_len = info->history ? (it < info->history_len ? it : info->history_len) : 0;
    return HX_OK;
}

// --------------------------------------------------------------- FGMRES
// Givens bookkeeping of one FGMRES cycle on the host: raw (unrotated)
// Hessenberg columns, rotations, rotated right-hand side g.
struct Hess {
    int m;
    std::vector<double> raw, R, cs, sn, g;
    explicit Hess(int m_) : m(m_), raw((size_t)(m_ + 1) * m_), R((size_t)(m_ + 1) * m_), cs(m_),
                            sn(m_), g(m_ + 1) {}
    double &h(int i, int j) { return raw[(size_t)i * m + j]; }
    double &r(int i, int j) { return R[(size_t)i * m + j]; }
    void reset(double beta)
    {
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
    }
    // rotate column j (entries 0..j+1 of raw) into R; false on breakdown
    bool rotate(int j)
    {
        for (int i = 0; i <= j + 1; ++i) r(i, j) = h(i, j);
        for (int i = 0; i < j; ++i) {
            const double t = cs[i] * r(i, j) + sn[i] * r(i + 1, j);
            r(i + 1, j) = -sn[i] * r(i, j) + cs[i] * r(i + 1, j);
            r(i, j) = t;
        }
        const double den = std::hypot(r(j, j), r(j + 1, j));
        if (!(den > 0.0) || !std::isfinite(den)) return false;
        cs[j] = r(j, j) / den;
        sn[j] = r(j + 1, j) / den;
        r(j, j) = den;
        r(j + 1, j) = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        return true;
    }
    // |g_{j+1}| that rotate(j) would give, without changing the state
    double peek(int j)
    {
        std::vector<double> col(j + 2);
        for (int i = 0; i <= j + 1; ++i) col[i] = h(i, j);
        for (int i = 0; i < j; ++i) {
            const double t = cs[i] * col[i] + sn[i] * col[i + 1];
            col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
            col[i] = t;
        }
        const double a = col[j], b = col[j + 1];
        const double den = std::hypot(a, b);
        if (!(den > 0.0) || !std::isfinite(den)) return INFINITY;
        return std::fabs(b / den * g[j]);
    }
};

// FGMRES(m), right preconditioned: A Z_k = V_{k+1} Hbar_k with orthonormal V
// and free Z (the preconditioner may change between steps).  Two ways of
// orthogonalising w = A z_j against V:
//  orth = 0: CGS2, two passes of block dot + update over V (four reads of V);
//  orth = 1: CGS2 with the second pass delayed by one step and fused with the
//    next step's pass: step j receives the once-orthogonalised, normalised
//    vector t_j, applies the preconditioner and A to it, and one block dot of
//    [V_{j-1}, t_j] against [t_j, w] gives both the reorthogonalisation
//    coefficients c of t_j and the projections of w.  One fused update then
//    finalises v_j = (t_j - V_{j-1} c)/rho and projects w (two reads of V).
//    Since t_j = rho v_j + V_{j-1} c, column j-1 of H gains nu_{j-1} c and
//    H(j, j-1) = nu_{j-1} rho one step late; a cycle ends with one extra
//    block dot that finalises its last column.  A step is one
//    preconditioner, one operator and three orthogonalisation launches
//    (partial block dots; their fixed-order sums and the step's scalars;
//    the fused update with partial sums of |w|^2), plus the normalisation
//    w/|w|, which block Jacobi folds into the next step's launch.  The
//    kernels write the step's scalars to pinned host memory themselves.
//    With a cheap preconditioner the host keeps one step in flight: it
//    launches step j+1 before it waits for the scalars of step j, and tests
//    convergence on the finalised columns.  With a costly one it runs one
//    step at a time and tests the provisional column first (its correction
//    is of the order of the loss of orthogonality), confirming after
//    finalising it.

hx_status solve_fgmres(hx_ctx *c, const hx_solve_params *prm, const double *b, double *x,
                       hx_solve_info *info, Timer &tm)
{
    const int64_t n = c->n_dofs;
    const int m = prm->restart;
    const size_t need64 = (size_t)(2 * m + 3) * n;
    const size_t need32 = prm->mixed ? 5 * (size_t)n : 0;
    hx_status s = ensure_work(c, need64, need32);
    if (s != HX_OK) return s;
    double *V = c->work64;                 // (m+1) n
    double *Z = V + (size_t)(m + 1) * n;   // m n
    double *w = Z + (size_t)m * n;         // n
    float *w32 = c->work32;
    // device scalars: [0..64] dots with the first vector, [64..128] with the
    // second, [128] |w|^2, [129] |b|^2, [130..194] y, [300..370] delayed step
    double *sc = c->red + SC_OFF;
    Hess H(m);
    std::vector<double> y(m);
    const bool delayed = prm->orth == 1;
    // delayed form: two steps in flight, slot j % 2 of the pinned buffer,
    // events and timers
    struct Ready {
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Ready()
        {
            for (auto &x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } rd;
    hipEvent_t *ready = rd.e;
    for (int i = 0; i < 2; ++i)
        if (hipEventCreateWithFlags(&ready[i], hipEventDisableTiming) != hipSuccess)
            return fail(c, HX_ERR_DEVICE, "hipEventCreate failed");
    Timer tb(tm.ok);
    Timer *tms[2] = {&tm, &tb};
    int nb_step[2] = {0, 0};
    double *fin_host = c->red_host;

    HX_HIP(c, blas_dot(c, n, b, b, sc + 129));
    double tmp[1];
    if ((s = read_scalars(c, sc + 129, 1, tmp)) != HX_OK) return s;
    const double nb = std::sqrt(tmp[0]);
    if (nb == 0.0) {
        HX_HIP(c, blas_fill(c, n, 0.0, x));
        info->true_rel_res = 0.0;
        return HX_OK;
    }
    if (prm->x0_mode != 1) HX_HIP(c, blas_fill(c, n, 0.0, x));
    int pc = prm->pc;
    int mixed = prm->mixed;
    int it = 0, hist = 0;
    std::vector<double> est_hist;
    bool done = false;
    // finalised residual estimate after column j: history, stall rule
    auto record = [&](int j) -> double {
        const double est = std::fabs(H.g[j + 1]) / nb;
        est_hist.push_back(est);
        if (info->history && hist < info->history_len) info->history[hist++] = est;
        return est;
    };
    auto stalled = [&]() {
        return pc == HX_PC_LEARNED && prm->stall_window > 0 &&
               (int)est_hist.size() > prm->stall_window &&
               est_hist.back() > prm->stall_ratio * est_hist[est_hist.size() - 1 - prm->stall_window];
    };
    // delayed form: reorthogonalise the tentative vector V[j+1] against
    // V[0..j] and finalise column j (H(0..j, j) += nu c, H(j+1, j) = nu rho)
    double nu_prev = 0.0;
    auto finalise = [&](int j) -> hx_status {
        tm.rec(2, c->stream);
        HX_HIP(c, blas_mdot(c, n, j + 2, V, n, V + (size_t)(j + 1) * n, sc));
        tm.rec(3, c->stream);
        HX_HIP(c, hipMemcpyAsync(fin_host, sc, sizeof(double) * (j + 2), hipMemcpyDeviceToHost,
                                 c->stream));
        HX_HIP(c, hipStreamSynchronize(c->stream));
        tm.orth += tm.span(2, 3);
        double cc = 0.0;
        for (int i = 0; i <= j; ++i) cc += fin_host[i] * fin_host[i];
        const double r2 = fin_host[j + 1] - cc;
        for (int i = 0; i <= j; ++i) H.h(i, j) += nu_prev * fin_host[i];
        H.h(j + 1, j) = r2 > 0.0 ? nu_prev * std::sqrt(r2) : 0.0;
        return HX_OK;
    };

    while (!done && it < prm->max_iter) {
        // explicit residual
        HX_HIP(c, sys_apply(c, prm, x, V, b));
        HX_HIP(c, blas_dot(c, n, V, V, sc + 128));
        if ((s = read_scalars(c, sc + 128, 1, tmp)) != HX_OK) return s;
        const double beta = std::sqrt(tmp[0]);
        const double rel0 = beta / nb;
        if (!std::isfinite(rel0)) return fail(c, HX_ERR_NOCONV, "non-finite residual");
        if (rel0 <= prm->rtol) break;
        HX_HIP(c, blas_scale_copy(c, n, sc + 128, 2, V, V));
        H.reset(beta);
        int j_used = 0;
        bool sw = false;
        for (int j = 0; !delayed && j < m && it < prm->max_iter; ++j) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            tm.rec(0, c->stream);
            if ((s = precondition(c, pc, mixed, prm->inner_iters, vj, zj, w32, &info->inner_iters)) != HX_OK)
                return s;
            tm.rec(1, c->stream);
            HX_HIP(c, step_apply(c, prm, zj, w, w32));
            tm.rec(2, c->stream);
            {
                // CGS2
                HX_HIP(c, blas_mdot(c, n, j + 1, V, n, w, sc));
                HX_HIP(c, blas_mupdate(c, n, j + 1, V, n, sc, -1.0, w));
                HX_HIP(c, blas_mdot(c, n, j + 1, V, n, w, sc + 64));
                HX_HIP(c, blas_mupdate(c, n, j + 1, V, n, sc + 64, -1.0, w));
                HX_HIP(c, blas_dot(c, n, w, w, sc + 128));
                HX_HIP(c, blas_scale_copy(c, n, sc + 128, 2, w, V + (size_t)(j + 1) * n));
                tm.rec(3, c->stream);
                HX_HIP(c, hipMemcpyAsync(c->red_host, sc, sizeof(double) * 129,
                                         hipMemcpyDeviceToHost, c->stream));
                HX_HIP(c, hipStreamSynchronize(c->stream));
                tm.acc();
                for (int i = 0; i <= j; ++i) H.h(i, j) = c->red_host[i] + c->red_host[64 + i];
                const double hn = std::sqrt(c->red_host[128]);
                H.h(j + 1, j) = hn;
                ++it;
                if (!H.rotate(j)) {
                    sw = true;
                    break;
                }
                j_used = j + 1;
                if (record(j) <= prm->rtol) break;
                if (stalled()) {
                    sw = true;
                    break;
                }
                if (!(hn > 0.0)) break;   // happy breakdown: exact solution in the space
                continue;
            }
        }
        // delayed CGS2, one step in flight: step j+1 is launched before the
        // host waits for the scalars of step j, so the stream never idles
        // while the host updates the Hessenberg matrix.  Step j+1 is what
        // finalises column j; when the cycle stops at column j it is
        // discarded (its column is never used).
        const int base = it;
        // cheap preconditioners run one step ahead; block Jacobi (also under
        // the learned correction) then takes the normalisation of the
        // previous step's w into its own launch.  Costly ones (inner FP32
        // CG, Chebyshev, multigrid) run one step at a time and test the
        // provisional column, so that no step is spent past convergence.
        const bool pipe = mixed != 1 && pc != HX_PC_CHEBYSHEV && pc != HX_PC_MULTIGRID &&
                          pc != HX_PC_MULTIGRID_MIXED;
        const bool fuse = pipe && !mixed && (pc == HX_PC_BLOCK_JACOBI || pc == HX_PC_LEARNED);
        auto will_launch = [&](int j) { return j < m && base + j < prm->max_iter; };
        int nb_prev = 0;   // partial sums of |w|^2 of the previous step
        auto launch_step = [&](int j) -> hx_status {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            Timer &t = *tms[j % 2];
            t.rec(0, c->stream);
            if (j > 0 && fuse) {
                if (pc == HX_PC_LEARNED) {
                    hx_status st = mlp_apply_fused(c, w, c->red + RED_WPART, nb_prev, vj, zj);
                    if (st != HX_OK) return st;
                } else {
                    HX_HIP(c, launch_bj64_scaled(c, w, c->red + RED_WPART, nb_prev, vj, zj));
                }
            } else {
                hx_status st = precondition(c, pc, mixed, prm->inner_iters, vj, zj, w32, &info->inner_iters);
                if (st != HX_OK) return st;
            }
            t.rec(1, c->stream);
            HX_HIP(c, step_apply(c, prm, zj, w, w32));
            t.rec(2, c->stream);
            const bool scale_now = !(fuse && will_launch(j + 1));
            HX_HIP(c, blas_dcgs(c, n, j, V, n, w, sc, c->pin_dev + (size_t)(j % 2) * FG_SLOT, scale_now,
                                &nb_prev));
            nb_step[j % 2] = nb_prev;
            t.rec(3, c->stream);
            HX_HIP(c, hipEventRecord(ready[j % 2], c->stream));
            return HX_OK;
        };
        for (int j = 0; delayed && will_launch(j); ++j) {
            if ((j == 0 || !pipe) && (s = launch_step(j)) != HX_OK) return s;
            const bool more = will_launch(j + 1);
            const bool ahead = pipe && more;
            if (ahead && (s = launch_step(j + 1)) != HX_OK) return s;
            if (hipEventSynchronize(ready[j % 2]) != hipSuccess)
                return fail(c, HX_ERR_DEVICE, "FGMRES: event wait failed");
            tms[j % 2]->acc();
            const double *hs = c->pin_host + (size_t)(j % 2) * FG_SLOT;
            const double rho = hs[DCGS_S + 2], hj = hs[DCGS_S + 3], flag = hs[DCGS_S + 4];
            const double nu = std::sqrt(host_sum256(hs + FG_PART, nb_step[j % 2]));
            ++it;
            if (j > 0) {
                // finalise column j-1 with the coefficients of t_j
                for (int i = 0; i < j; ++i) H.h(i, j - 1) += nu_prev * hs[i];
                H.h(j, j - 1) = flag != 0.0 ? 0.0 : nu_prev * rho;
                if (!H.rotate(j - 1)) {
                    sw = true;
                    break;
                }
                j_used = j;
                if (record(j - 1) <= prm->rtol) break;
                if (stalled()) {
                    sw = true;
                    break;
                }
                if (flag != 0.0) break;   // t_j in span(V): exact solution in the space
            } else if (flag != 0.0) {
                sw = true;   // the residual direction itself degenerated
                break;
            }
            if (!std::isfinite(nu) || !std::isfinite(hj)) {
                sw = true;
                break;
            }
            // provisional column j
            for (int i = 0; i < j; ++i) H.h(i, j) = hs[64 + i];
            H.h(j, j) = hj;
            H.h(j + 1, j) = nu;
            nu_prev = nu;
            if (!(nu > 0.0)) {
                // happy breakdown: the column is final as it stands
                if (!H.rotate(j)) {
                    sw = true;
                    break;
                }
                j_used = j + 1;
                record(j);
                break;
            }
            if (ahead) continue;   // step j+1, in flight, finalises column j
            if (!more || H.peek(j) / nb <= prm->rtol) {
                // last step of the cycle, or the provisional column passes:
                // finalise it here
                if ((s = finalise(j)) != HX_OK) return s;
                if (!H.rotate(j)) {
                    sw = true;
                    break;
                }
                j_used = j + 1;
                if (record(j) <= prm->rtol || !more) break;
                if (stalled()) {
                    sw = true;
                    break;
                }
                // not converged after all: the next step recomputes the same
                // coefficients and adds them to the now-final column, so undo
                for (int i = 0; i <= j; ++i) H.h(i, j) = i < j ? hs[64 + i] : hj;
                H.h(j + 1, j) = nu;
                H.g[j] = H.cs[j] * H.g[j] - H.sn[j] * H.g[j + 1];
                H.g[j + 1] = 0.0;
                est_hist.pop_back();
                if (info->history && hist > 0) --hist;
                j_used = j;
            }
        }
        if (j_used > 0) {
            for (int i = j_used - 1; i >= 0; --i) {
                double t = H.g[i];
                for (int k = i + 1; k < j_used; ++k) t -= H.r(i, k) * y[k];
                y[i] = t / H.r(i, i);
            }
            HX_HIP(c, hipMemcpyAsync(sc + 130, y.data(), sizeof(double) * j_used,
                                     hipMemcpyHostToDevice, c->stream));
            HX_HIP(c, blas_lincomb(c, n, j_used, Z, n, sc + 130, x));
        }
        ++info->restarts;
        if (sw) {
            if (pc == HX_PC_LEARNED) {
                pc = HX_PC_BLOCK_JACOBI;
                info->fallback_used = 1;
                est_hist.clear();
            } else {
                done = true;   // breakdown with no fallback left
            }
        }
    }
    tm.op += tb.op;
    tm.pc += tb.pc;
    tm.orth += tb.orth;
    info->iters = it;
    info->history_len = info->history ? hist : 0;
    return HX_OK;
}

}  // namespace

// Chebyshev polynomial preconditioner (section 3.1 names it for the SPD
// systems: a polynomial in M^-1 A that damps the eigenvalue range, the range
// estimated by the Lanczos process; M = block Jacobi).  degree steps of the
// Chebyshev iteration for A z = r from z = 0 (or from a given z, the same
// polynomial acting on the error) on [lo, hi]:
//   d = M^-1 (r - A z) / theta, z += d; then rho' = 1/(2 sigma - rho),
//   d = rho' rho d + (2 rho' / delta) M^-1 (r - A z), z += d,
// theta = (hi + lo)/2, delta = (hi - lo)/2, sigma = theta/delta, rho = 1/sigma.
hipError_t cheb_iterate64(hx_ctx *c, const double *b, double *x, bool x_zero)
{
    const int64_t n = c->n_dofs;
    double *res = c->chebw, *d = res + n;
    const double theta = 0.5 * (c->cheb_hi + c->cheb_lo), delta = 0.5 * (c->cheb_hi - c->cheb_lo);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    hipError_t e = hipSuccess;
    const double *v = b;
    if (!x_zero) {
        e = launch_apply64(c, x, res, b);                       // res = b - A x
        v = res;
    }
    // d = M^-1 v / theta; x = d or x += d (the block-Jacobi kernel's epilogue)
    if (e == hipSuccess) e = launch_bj_cheb64(c, v, d, x, 1.0 / theta, 0.0, 0, !x_zero);
    for (int k = 1; k < c->cheb_deg && e == hipSuccess; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        e = launch_apply64(c, x, res, b);                       // res = b - A x
        if (e == hipSuccess) e = launch_bj_cheb64(c, res, d, x, 2.0 * rn / delta, rn * rho, 1, 1);
        rho = rn;
    }
    return e;
}

hipError_t cheb_apply64(hx_ctx *c, const double *r, double *z) { return cheb_iterate64(c, r, z, true); }

hipError_t cheb_iterate32(hx_ctx *c, const float *b, float *x, bool x_zero)
{
    const int64_t n = c->n_dofs;
    float *res = c->chebw32, *d = res + n;
    const double theta = 0.5 * (c->cheb_hi + c->cheb_lo), delta = 0.5 * (c->cheb_hi - c->cheb_lo);
    const double sigma = theta / delta;
    double rho = 1.0 / sigma;
    hipError_t e = hipSuccess;
    const float *v = b;
    if (!x_zero) {
        e = launch_apply32(c, x, res, b);
        v = res;
    }
    if (e == hipSuccess) e = launch_bj_cheb32(c, v, d, x, 1.0 / theta, 0.0, 0, !x_zero);
    for (int k = 1; k < c->cheb_deg && e == hipSuccess; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        e = launch_apply32(c, x, res, b);
        if (e == hipSuccess) e = launch_bj_cheb32(c, res, d, x, 2.0 * rn / delta, rn * rho, 1, 1);
        rho = rn;
    }
    return e;
}

hx_status mg_check(hx_ctx *c)
{
    int depth = 0;
    for (hx_ctx *L = c; L; L = L->mg_coarse, ++depth) {
        if (!L->has_coef) return fail(c, HX_ERR_STATE, "multigrid level %d has no coefficients", depth);
        if (L->cheb_deg < 1)
            return fail(c, HX_ERR_STATE, "multigrid level %d has no Chebyshev smoother", depth);
        if (L->mg_coarse) {
            const hx_ctx *C = L->mg_coarse;
            if (!L->mgw || !C->mgw || !L->mgw32 || !C->mgw32 || C->n_cells != L->mg_nc ||
                C->k != L->k || C->stream != L->stream)
                return fail(c, HX_ERR_STATE,
                            "multigrid level %d changed since hx_set_multigrid; link it again", depth + 1);
        }
    }
    return HX_OK;
}

}  // namespace hx

using namespace hx;

extern "C" {

void hx_default_params(hx_solve_params *p)
{
    if (!p) return;
    p->method = 0;
    p->restart = 30;
    p->rtol = 1e-8;
    p->max_iter = 10000;
    p->pc = HX_PC_BLOCK_JACOBI;
    p->mixed = 0;
    p->inner_iters = 32;
    p->inner_rtol = 1e-2;
    p->x0_mode = 0;
    p->stall_window = 10;
    p->stall_ratio = 0.99;
    p->orth = 1;
    p->system = 0;
}

hx_status hx_solve(hx_ctx *c, const hx_solve_params *prm, const double *b, double *x,
                   hx_solve_info *info)
{
    if (!c) return HX_ERR_ARG;
    if (!prm || !b || !x || !info) return fail(c, HX_ERR_ARG, "null argument");
    double *hist = info->history;
    int hcap = info->history_len;
    std::memset(info, 0, sizeof(*info));
    info->history = hist;
    info->history_len = hist ? hcap : 0;
    info->status = HX_ERR_STATE;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "solve before setup_mesh/set_coefficients");
    if (b == x) return fail(c, HX_ERR_ARG, "b and x alias");
    if (prm->method != 0 && prm->method != 1) return fail(c, HX_ERR_ARG, "method must be 0 or 1");
    if (prm->method == 1 && (prm->restart < 1 || prm->restart > 63))
        return fail(c, HX_ERR_ARG, "restart must be in 1..63");
    if (prm->orth != 0 && prm->orth != 1) return fail(c, HX_ERR_ARG, "orth must be 0 or 1");
    if (!(prm->rtol > 0.0) || prm->max_iter < 1) return fail(c, HX_ERR_ARG, "bad rtol/max_iter");
    if (prm->pc < HX_PC_NONE || prm->pc > HX_PC_MULTIGRID_MIXED) return fail(c, HX_ERR_ARG, "bad pc");
    if (prm->method == 0 && (prm->pc == HX_PC_LEARNED || prm->mixed))
        return fail(c, HX_ERR_ARG, "CG needs a fixed SPD preconditioner; use FGMRES");
    if (prm->mixed < 0 || prm->mixed > 2) return fail(c, HX_ERR_ARG, "mixed must be 0, 1 or 2");
    if (prm->mixed == 1 && prm->inner_iters < 1) return fail(c, HX_ERR_ARG, "inner_iters must be >= 1");
    if (prm->mixed == 2 && prm->system != 0)
        return fail(c, HX_ERR_ARG, "the minimal mixed form has an FP32 operator only for the Helmholtz-type system");
    if (prm->mixed && prm->pc == HX_PC_LEARNED)
        return fail(c, HX_ERR_ARG, "the learned preconditioner is FP64; it cannot precondition the inner FP32 solve");
    if (prm->pc == HX_PC_LEARNED && !c->mlp) return fail(c, HX_ERR_STATE, "no network loaded");
    if (prm->pc == HX_PC_CHEBYSHEV && c->cheb_deg < 1)
        return fail(c, HX_ERR_STATE, "Chebyshev preconditioner not set");
    if (prm->pc == HX_PC_CHEBYSHEV && prm->mixed)
        return fail(c, HX_ERR_ARG, "the Chebyshev preconditioner is FP64; it cannot precondition the inner FP32 solve");
    const bool mgpc = prm->pc == HX_PC_MULTIGRID || prm->pc == HX_PC_MULTIGRID_MIXED;
    if (mgpc && prm->mixed)
        return fail(c, HX_ERR_ARG, "the multigrid preconditioner works on FP64 residuals; it cannot precondition the inner FP32 solve");
    if (mgpc) {
        const hx_status s = mg_check(c);
        if (s != HX_OK) return s;
    }
    if (prm->system < 0 || prm->system > 2) return fail(c, HX_ERR_ARG, "system must be 0, 1 or 2");
    if (prm->system == 2 && !c->has_q) return fail(c, HX_ERR_STATE, "consistent integration not set");
    if (prm->system == 1 && !c->has_press) return fail(c, HX_ERR_STATE, "pressure system not set");
    if (prm->system == 1 && prm->method != 1)
        return fail(c, HX_ERR_ARG, "the pressure system is not symmetric; use FGMRES");
    HX_HIP(c, hipSetDevice(c->device));
    const double t0 = now_ms();
    Timer tm(true);
    hx_status s = prm->method == 0 ? solve_cg(c, prm, b, x, info, tm)
                                   : solve_fgmres(c, prm, b, x, info, tm);
    if (s != HX_OK && s != HX_ERR_NOCONV) {
        info->status = s;
        return s;
    }
    // the true FP64 residual decides
    const int64_t n = c->n_dofs;
    double *sc = c->red + SC_OFF;
    hx_status s2 = ensure_work(c, (size_t)n, 0);
    if (s2 != HX_OK) return s2;
    HX_HIP(c, sys_apply(c, prm, x, c->work64, b));
    HX_HIP(c, blas_dot(c, n, c->work64, c->work64, sc + 200));
    HX_HIP(c, blas_dot(c, n, b, b, sc + 201));
    double hh[2];
    if ((s2 = read_scalars(c, sc + 200, 2, hh)) != HX_OK) return s2;
    info->true_rel_res = hh[1] > 0 ? std::sqrt(hh[0] / hh[1]) : 0.0;
    info->ms_total = now_ms() - t0;
    info->ms_op = tm.op;
    info->ms_pc = tm.pc;
    info->ms_orth = tm.orth;
    const bool conv = info->true_rel_res <= prm->rtol * 1.0001;
    hx_status st = conv ? (info->fallback_used ? HX_FALLBACK_USED : HX_OK) : HX_ERR_NOCONV;
    info->status = st;
    if (st == HX_ERR_NOCONV)
        fail(c, st, "not converged: true relative residual %.3e after %d iterations",
             info->true_rel_res, info->iters);
    return st;
}


hx_status hx_solve_pressure_fixed_point(hx_ctx *c, const double *rho, const double *F,
                                        const double *G, double *p, double gamma, double tau,
                                        double penalty_factor, const hx_solve_params *prm,
                                        int max_fp_iters, double fp_tol, int *fp_iters,
                                        double *fp_change, hx_solve_info *info)
{
    if (!c) return HX_ERR_ARG;
    if (!rho || !F || !G || !p || !prm || !info) return fail(c, HX_ERR_ARG, "null argument");
    if (!c->has_mesh) return fail(c, HX_ERR_STATE, "fixed point before setup_mesh");
    if (max_fp_iters < 1 || !(fp_tol > 0.0)) return fail(c, HX_ERR_ARG, "bad fixed-point limits");
    if (prm->method != 1) return fail(c, HX_ERR_ARG, "the pressure system needs FGMRES");
    HX_HIP(c, hipSetDevice(c->device));
    const int64_t n = c->n_dofs;
    double *tmp = nullptr;      // h, rhs, p_new
    hx_status s = dalloc(c, (void **)&tmp, sizeof(double) * 3 * n);
    if (s != HX_OK) return s;
    double *h = tmp, *rhs = tmp + n, *pn = tmp + 2 * n;
    double *sc = c->red + SC_OFF + 300;
    hx_solve_params q = *prm;
    q.system = 1;
    q.x0_mode = 1;
    int it = 0;
    double change = 0.0;
    bool conv = false, lin_ok = true;
    for (it = 0; it < max_fp_iters && !conv; ++it) {
        hipError_t e = launch_enthalpy(c, p, rho, gamma, h);
        if (e != hipSuccess) { s = fail(c, HX_ERR_DEVICE, "enthalpy: %s", hipGetErrorString(e)); break; }
        if ((s = hx_set_pressure_system(c, rho, h, gamma, tau, penalty_factor, 1)) != HX_OK) break;
        if ((s = hx_pressure_rhs(c, F, G, rhs)) != HX_OK) break;
        e = hipMemcpyAsync(pn, p, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) { s = fail(c, HX_ERR_DEVICE, "copy: %s", hipGetErrorString(e)); break; }
        s = hx_solve(c, &q, rhs, pn, info);
        if (s != HX_OK && s != HX_FALLBACK_USED && s != HX_ERR_NOCONV) break;
        lin_ok = s != HX_ERR_NOCONV;
        s = HX_OK;
        // change = ||p_new - p|| / ||p_new||; then p = p_new
        e = blas_axpby(c, n, 1.0, pn, -1.0, p);
        if (e == hipSuccess) e = blas_dot(c, n, p, p, sc);
        if (e == hipSuccess) e = blas_dot(c, n, pn, pn, sc + 1);
        if (e == hipSuccess) e = hipMemcpyAsync(p, pn, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) { s = fail(c, HX_ERR_DEVICE, "update: %s", hipGetErrorString(e)); break; }
        double hh[2];
        if ((s = read_scalars(c, sc, 2, hh)) != HX_OK) break;
        change = hh[1] > 0.0 ? std::sqrt(hh[0] / hh[1]) : std::sqrt(hh[0]);
        conv = change <= fp_tol;
    }
    dfree((void **)&tmp);
    if (fp_iters) *fp_iters = it;
    if (fp_change) *fp_change = change;
    if (s != HX_OK) return s;
    if (!conv || !lin_ok)
        return fail(c, HX_ERR_NOCONV, "fixed point: change %.3e after %d iterations%s", change, it,
                    lin_ok ? "" : " (last linear solve not converged)");
    return HX_OK;
}


hx_status hx_set_chebyshev(hx_ctx *c, int degree, double lo, double hi)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "set_chebyshev before set_coefficients");
    if (degree < 1 || degree > 64) return fail(c, HX_ERR_ARG, "degree must be in 1..64");
    if (!(lo > 0.0) || !(hi > lo) || !std::isfinite(hi)) return fail(c, HX_ERR_ARG, "need 0 < lo < hi");
    HX_HIP(c, hipSetDevice(c->device));
    if (!c->chebw) {
        hx_status s = dalloc(c, (void **)&c->chebw, sizeof(double) * 2 * c->n_dofs);
        if (s == HX_OK) s = dalloc(c, (void **)&c->chebw32, sizeof(float) * 2 * c->n_dofs);
        if (s != HX_OK) return s;
    }
    c->cheb_deg = degree;
    c->cheb_lo = lo;
    c->cheb_hi = hi;
    return HX_OK;
}

hx_status hx_set_multigrid(hx_ctx *c, hx_ctx *coarse, const int32_t *parent, const int32_t *octant)
{
    if (!c) return HX_ERR_ARG;
    HX_HIP(c, hipSetDevice(c->device));
    dfree((void **)&c->mg_cptr);
    dfree((void **)&c->mg_clist);
    dfree((void **)&c->mg_child8);
    c->mg_coarse = nullptr;
    c->mg_nc = 0;
    if (!coarse) return HX_OK;
    if (c->n_hang || coarse->n_hang)
        return fail(c, HX_ERR_STATE, "multigrid levels are uniform refinements; this mesh has hanging faces");
    if (!c->has_mesh || !coarse->has_mesh) return fail(c, HX_ERR_STATE, "set_multigrid before setup_mesh");
    if (!parent || !octant) return fail(c, HX_ERR_ARG, "parent and octant are required");
    if (coarse->device != c->device || coarse->stream != c->stream)
        return fail(c, HX_ERR_ARG, "the levels must share the device and the stream");
    if (coarse->k != c->k) return fail(c, HX_ERR_ARG, "the levels must have the same degree");
    for (const hx_ctx *p = coarse; p; p = p->mg_coarse)
        if (p == c) return fail(c, HX_ERR_ARG, "the levels would form a cycle");
    const int64_t nf = c->n_cells, nc = coarse->n_cells;
    if (nf >= (int64_t(1) << 28)) return fail(c, HX_ERR_ARG, "too many cells for the child list");
    std::vector<int32_t> ptr(nc + 1, 0), list(nf);
    std::vector<uint8_t> used(nc, 0);
    for (int64_t f = 0; f < nf; ++f) {
        const int32_t p = parent[f], o = octant[f];
        if (p < 0 || p >= nc || o < 0 || o > 7)
            return fail(c, HX_ERR_ARG, "cell %lld: parent %d or octant %d out of range", (long long)f, p, o);
        if (used[p] >> o & 1)
            return fail(c, HX_ERR_ARG, "cell %lld: octant %d of parent %d already taken", (long long)f, o, p);
        used[p] |= (uint8_t)(1u << o);
        ++ptr[p + 1];
    }
    for (int64_t j = 0; j < nc; ++j) ptr[j + 1] += ptr[j];
    {
        std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t f = 0; f < nf; ++f) list[fill[parent[f]]++] = (int32_t)(f * 8 + octant[f]);
    }
    hx_status s = dalloc(c, (void **)&c->mg_cptr, sizeof(int32_t) * (nc + 1));
    if (s == HX_OK) s = dalloc(c, (void **)&c->mg_clist, sizeof(int32_t) * nf);
    for (hx_ctx *L : {c, coarse})
        if (s == HX_OK && !L->mgw) {
            s = dalloc(L, (void **)&L->mgw, sizeof(double) * 3 * L->n_dofs);
            if (s == HX_OK) s = dalloc(L, (void **)&L->mgw32, sizeof(float) * 3 * L->n_dofs);
        }
    if (s != HX_OK) return s;
    HX_HIP(c, hipMemcpy(c->mg_cptr, ptr.data(), sizeof(int32_t) * (nc + 1), hipMemcpyHostToDevice));
    HX_HIP(c, hipMemcpy(c->mg_clist, list.data(), sizeof(int32_t) * nf, hipMemcpyHostToDevice));
    // every coarse cell with all eight children: the octant table of the
    // dense transfer kernels
    bool full = nf == 8 * nc;
    for (int64_t j = 0; full && j < nc; ++j) full = used[j] == 0xFF;
    if (full) {
        std::vector<int32_t> c8((size_t)8 * nc);
        for (int64_t f = 0; f < nf; ++f) c8[(size_t)8 * parent[f] + octant[f]] = (int32_t)f;
        if ((s = dalloc(c, (void **)&c->mg_child8, sizeof(int32_t) * 8 * nc)) != HX_OK) return s;
        HX_HIP(c, hipMemcpy(c->mg_child8, c8.data(), sizeof(int32_t) * 8 * nc, hipMemcpyHostToDevice));
    }
    c->mg_coarse = coarse;
    c->mg_nc = nc;
    return HX_OK;
}

hx_status hx_mg_transfer(hx_ctx *c, int dir, const double *in, double *out)
{
    if (!c) return HX_ERR_ARG;
    if (!c->mg_coarse) return fail(c, HX_ERR_STATE, "no coarser level set");
    if (dir != 0 && dir != 1) return fail(c, HX_ERR_ARG, "dir must be 0 (restrict) or 1 (prolong)");
    if (!in || !out || in == out) return fail(c, HX_ERR_ARG, "bad vectors");
    if (c->mg_coarse->n_cells != c->mg_nc || !c->mg_coarse->has_mesh)
        return fail(c, HX_ERR_STATE, "the coarser level changed since hx_set_multigrid");
    HX_HIP(c, hipSetDevice(c->device));
    if (dir == 0) HX_HIP(c, mg_restrict64(c, in, out));
    else HX_HIP(c, mg_prolong_add64(c, in, out));
    return HX_OK;
}

hx_status hx_estimate_eigenvalues(hx_ctx *c, const double *b, int iters, double *lo, double *hi)
{
    if (!c) return HX_ERR_ARG;
    if (!c->has_coef) return fail(c, HX_ERR_STATE, "estimate before set_coefficients");
    if (!b || !lo || !hi || iters < 1 || iters > 200) return fail(c, HX_ERR_ARG, "bad arguments");
    HX_HIP(c, hipSetDevice(c->device));
    const int64_t n = c->n_dofs;
    hx_status s = ensure_work(c, 4 * (size_t)n, 0);
    if (s != HX_OK) return s;
    double *r = c->work64, *z = r + n, *p = z + n, *q = p + n;
    double *sc = c->red + SC_OFF + 310;
    HX_HIP(c, blas_copy(c, n, b, r));
    HX_HIP(c, launch_bj64(c, r, z));
    HX_HIP(c, blas_copy(c, n, z, p));
    HX_HIP(c, blas_dot(c, n, r, z, sc));
    double rz;
    if ((s = read_scalars(c, sc, 1, &rz)) != HX_OK) return s;
    std::vector<double> al, ga;
    for (int k = 0; k < iters && rz > 0.0; ++k) {
        double pq, rzn;
        HX_HIP(c, launch_apply64(c, p, q, nullptr));
        HX_HIP(c, blas_dot(c, n, p, q, sc + 1));
        if ((s = read_scalars(c, sc + 1, 1, &pq)) != HX_OK) return s;
        if (!(pq > 0.0)) break;
        const double a = rz / pq;
        HX_HIP(c, blas_axpby(c, n, -a, q, 1.0, r));
        HX_HIP(c, launch_bj64(c, r, z));
        HX_HIP(c, blas_dot(c, n, r, z, sc + 2));
        if ((s = read_scalars(c, sc + 2, 1, &rzn)) != HX_OK) return s;
        const double g = rzn / rz;
        al.push_back(a);
        ga.push_back(g);
        HX_HIP(c, blas_axpby(c, n, 1.0, z, g, p));
        rz = rzn;
    }
    const int m = (int)al.size();
    if (m < 1) return fail(c, HX_ERR_ARG, "no Lanczos step possible");
    // Lanczos tridiagonal matrix from the CG coefficients, dense for sym_eig
    std::vector<double> T((size_t)m * m, 0.0), w(m), v((size_t)m * m);
    for (int k = 0; k < m; ++k) {
        T[(size_t)k * m + k] = 1.0 / al[k] + (k > 0 ? ga[k - 1] / al[k - 1] : 0.0);
        if (k + 1 < m) T[(size_t)k * m + k + 1] = T[(size_t)(k + 1) * m + k] = std::sqrt(ga[k]) / al[k];
    }
    sym_eig(m, T.data(), w.data(), v.data());
    double mn = w[0], mx = w[0];
    for (int k = 1; k < m; ++k) {
        mn = std::min(mn, w[k]);
        mx = std::max(mx, w[k]);
    }
    *lo = mn;
    *hi = mx;
    return HX_OK;
}

}  // extern "C"
