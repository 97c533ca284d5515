// Separable cell-block Jacobi by fast diagonalisation:
//   z_K = (S_z (x) S_y (x) S_x) diag(1/(c0 + cx lx_i + cy ly_j + cz lz_l))
//         (S_z (x) S_y (x) S_x)^T r_K,
// with S_d^T M S_d = I and S_d^T L_d S_d = diag(l_d) per cell and direction.
// This is the tensor-product inversion of block-diagonal operators the paper
// uses for its velocity mass matrix (section 3.3: inverse as S^-T J^-1 S^-1
// with S a Kronecker product of 1-D matrices), applied here to the
// separable approximation of the Helmholtz cell block.
//
// Mapping: N*N threads per cell, one per pencil; 6 sweeps of N x N 1-D
// matrices that differ per cell (kept in LDS) plus one diagonal scaling.
// A fused form also performs the conjugate-gradient updates of x and r
// before the solve and sums r.z and r.r per block, so one CG step touches
// each vector once.
#include "common.hpp"
#include "bj_cell.hpp"
#include "sum256.hpp"

#include <cstddef>
#include <type_traits>

namespace hx {

namespace {

template <int N>
struct Cfg {
    static constexpr int NF = N * N, ND = N * N * N;
    static constexpr int CPB = (256 / NF) > 0 ? 256 / NF : 1;
    static constexpr int NT = ((CPB * NF + 63) / 64) * 64;
};

// deterministic block sum of two values (result valid in thread 0)
template <int NT>
__device__ __forceinline__ void block_sum2(double &u, double &v, double *sh)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        u += __shfl_down(u, o, 64);
        v += __shfl_down(v, o, 64);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) {
        sh[2 * wv] = u;
        sh[2 * wv + 1] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        u = v = 0.0;
        for (int i = 0; i < NT / 64; ++i) {
            u += sh[2 * i];
            v += sh[2 * i + 1];
        }
    }
}

// FUSE: one conjugate-gradient step around the preconditioner, with the
// step length a = sc[0] / sc[1] (r.z over p.q) read from device memory (0
// when p.q is exactly 0: a step in flight after exact convergence):
//   x += a p,  r -= a q,  z = M^{-1} r,
// and per-block partial sums of r.z and r.r written to part[blk] and
// part[ld + blk].  CHEB: one step of the Chebyshev iteration around the
// preconditioner, z holding the step direction d and x the iterate:
//   d = ca M^{-1} r + cb d  (cb read only with CHEB_READ_D),
//   x = x + d  (CHEB_ACCUM)  or  x = d.
// Otherwise plain z = M^{-1} r, or, with part given (scaled form: ld
// partial sums of |r|^2 in part), z = M^{-1} (r / |r|) and x = r / |r|, the
// norm from the fixed-order sum256 of the partial sums.
constexpr int CHEB_READ_D = 1, CHEB_ACCUM = 2;

template <int N, typename T, bool FUSE, bool CHEB = false>
__global__ void __launch_bounds__(Cfg<N>::NT)
k_bj(const T *__restrict__ rin, T *__restrict__ z, const T *__restrict__ S, const T *__restrict__ L,
     const T *__restrict__ C, int n_cells, int nwg, T *x, T *rw, const T *__restrict__ p,
     const T *__restrict__ q, const double *__restrict__ sc, double *part, int ld, T ca = 0,
     T cb = 0, int flags = 0, const double *__restrict__ pqp = nullptr, int npq = 0)
{
    const T *r = FUSE ? rw : rin;
    constexpr int NF = Cfg<N>::NF, ND = Cfg<N>::ND, CPB = Cfg<N>::CPB;
    __shared__ T sR[CPB][ND];
    __shared__ T sS[CPB][3][NF];
    __shared__ T sL[CPB][3][N];
    __shared__ T sC[CPB][4];

    const int bid = blockIdx.x;
    const int q8 = nwg / NXCD, r8 = nwg % NXCD, xcd = bid % NXCD;
    const int wg = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / NXCD;
    const int t = threadIdx.x;
    const int lc0 = t / NF;
    const bool slot = lc0 < CPB;
    const int lc = slot ? lc0 : 0;
    const int tt = t - lc0 * NF;
    const int a = tt % N, b = tt / N;
    const int64_t cid = (int64_t)wg * CPB + lc;
    const bool active = slot && cid < n_cells;

    double acc_rr = 0.0, acc_rz = 0.0;
    T sfac = 1;
    const bool scaled = !FUSE && !CHEB && part != nullptr;
    if (scaled) {
        static_assert(Cfg<N>::NT == 256, "the scaled form sums with a 256-thread workgroup");
        __shared__ double shs[4];
        sfac = (T)(1.0 / sqrt(sum256(part, ld, shs)));
    }
    // p.q: the operator's partial sums summed here (every workgroup the same
    // fixed order), or the value in sc[1]
    double pq = 0.0;
    if (FUSE) {
        if (pqp) {
            __shared__ double shq[4];
            pq = sum256(pqp, npq, shq);
        } else {
            pq = sc[1];
        }
    }
    // every global load of the cell at once (one memory round trip): the
    // residual (and for the CG step x, p and q), the eigenvector matrices,
    // the eigenvalues and the constants; each thread's values lie NF apart
    constexpr int NLS = (3 * N + NF - 1) / NF;   // eigenvalue loads per thread
    T rv[N], xv[N], pv[N], qv[N], tS[3], tL[NLS], tC = 0;
    if (active) {
        const T *rs = FUSE ? rw : r;
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const int64_t gi = cid * ND + tt + u * NF;
            rv[u] = rs[gi];
            if (FUSE) {
                xv[u] = x[gi];
                pv[u] = p[gi];
                qv[u] = q[gi];
            }
        }
#pragma unroll
        for (int u = 0; u < 3; ++u) tS[u] = S[cid * 3 * NF + tt + u * NF];
#pragma unroll
        for (int u = 0; u < NLS; ++u) {
            const int e = tt + u * NF;
            tL[u] = e < 3 * N ? L[cid * 3 * N + e] : T(0);
        }
        if (tt < 4) tC = C[cid * 4 + tt];
    }
    // (the scheduler would otherwise wait for each load before the next)
    __builtin_amdgcn_sched_barrier(0);
    if (FUSE && active) {
        const T al = (T)(pq != 0.0 ? sc[0] / pq : 0.0);
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const int e = tt + u * NF;
            const int64_t gi = cid * ND + e;
            const T rn = rv[u] - al * qv[u];
            x[gi] = xv[u] + al * pv[u];
            rw[gi] = rn;
            sR[lc][e] = rn;
            acc_rr += (double)rn * (double)rn;
        }
    } else if (active && scaled) {
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const int e = tt + u * NF;
            const T rn = rv[u] * sfac;
            x[cid * ND + e] = rn;
            sR[lc][e] = rn;
        }
    } else if (active) {
#pragma unroll
        for (int u = 0; u < N; ++u) sR[lc][tt + u * NF] = rv[u];
    }
    if (active) {
#pragma unroll
        for (int u = 0; u < 3; ++u) sS[lc][u][tt] = tS[u];
#pragma unroll
        for (int u = 0; u < NLS; ++u) {
            const int e = tt + u * NF;
            if (e < 3 * N) sL[lc][e / N][e % N] = tL[u];
        }
        if (tt < 4) sC[lc][tt] = tC;
    }
    __syncthreads();
    bj_cell_solve<N, T>(sR[lc], sS[lc], sL[lc], sC[lc], a, b, active, acc_rz);
    if (active) {
        if (CHEB) {
            T zo[N], xo[N];
#pragma unroll
            for (int u = 0; u < N; ++u) {
                const int64_t gi = cid * ND + tt + u * NF;
                zo[u] = (flags & CHEB_READ_D) ? z[gi] : T(0);
                xo[u] = (flags & CHEB_ACCUM) ? x[gi] : T(0);
            }
#pragma unroll
            for (int u = 0; u < N; ++u) {
                const int e = tt + u * NF;
                const int64_t gi = cid * ND + e;
                T dn = ca * sR[lc][e];
                if (flags & CHEB_READ_D) dn += cb * zo[u];
                z[gi] = dn;
                x[gi] = (flags & CHEB_ACCUM) ? xo[u] + dn : dn;
            }
        } else {
#pragma unroll
            for (int u = 0; u < N; ++u) z[cid * ND + tt + u * NF] = sR[lc][tt + u * NF];
        }
    }
    if (FUSE) {
        __shared__ double sh2[2 * (Cfg<N>::NT / 64)];
        block_sum2<Cfg<N>::NT>(acc_rz, acc_rr, sh2);
        if (threadIdx.x == 0) {
            part[bid] = acc_rz;
            part[ld + bid] = acc_rr;
        }
    }
}

// CG step arguments of the fused form (null for a plain application)
template <typename T>
struct CgArgs {
    T *x = nullptr, *r = nullptr;
    const T *p = nullptr, *q = nullptr;
    const double *sc = nullptr;
    const double *pqp = nullptr;   // partial sums of p.q (null: p.q in sc[1])
    int npq = 0;
};

template <int N, typename T>
hipError_t bj_cheb_n(hx_ctx *c, const T *r, T *d, T *x, double ca, double cb, int flags)
{
    const int cpb = Cfg<N>::CPB;
    const int nwg = (int)((c->n_cells + cpb - 1) / cpb);
    const bool dbl = std::is_same<T, double>::value;
    const T *S = dbl ? (const T *)c->bjS64 : (const T *)c->bjS32;
    const T *L = dbl ? (const T *)c->bjL64 : (const T *)c->bjL32;
    const T *C = dbl ? (const T *)c->bjC64 : (const T *)c->bjC32;
    hipLaunchKernelGGL((k_bj<N, T, false, true>), dim3(nwg), dim3(Cfg<N>::NT), 0, c->stream, r, d,
                       S, L, C, (int)c->n_cells, nwg, x, (T *)nullptr, (const T *)nullptr,
                       (const T *)nullptr, (const double *)nullptr, (double *)nullptr, 0, (T)ca,
                       (T)cb, flags);
    return hipGetLastError();
}

template <typename T>
hipError_t bj_cheb_dispatch(hx_ctx *c, const T *r, T *d, T *x, double ca, double cb, int read_d,
                            int accum)
{
    const int flags = (read_d ? CHEB_READ_D : 0) | (accum ? CHEB_ACCUM : 0);
    switch (c->n) {
    case 2: return bj_cheb_n<2, T>(c, r, d, x, ca, cb, flags);
    case 3: return bj_cheb_n<3, T>(c, r, d, x, ca, cb, flags);
    case 4: return bj_cheb_n<4, T>(c, r, d, x, ca, cb, flags);
    case 5: return bj_cheb_n<5, T>(c, r, d, x, ca, cb, flags);
    case 6: return bj_cheb_n<6, T>(c, r, d, x, ca, cb, flags);
    case 7: return bj_cheb_n<7, T>(c, r, d, x, ca, cb, flags);
    case 8: return bj_cheb_n<8, T>(c, r, d, x, ca, cb, flags);
    default: return hipErrorInvalidValue;
    }
}

template <int N, typename T>
hipError_t bj_n(hx_ctx *c, const T *r, T *z, const CgArgs<T> *cg, int *nblk)
{
    const int cpb = Cfg<N>::CPB;
    const int nwg = (int)((c->n_cells + cpb - 1) / cpb);
    const bool dbl = std::is_same<T, double>::value;
    const T *S = dbl ? (const T *)c->bjS64 : (const T *)c->bjS32;
    const T *L = dbl ? (const T *)c->bjL64 : (const T *)c->bjL32;
    const T *C = dbl ? (const T *)c->bjC64 : (const T *)c->bjC32;
    if (nblk) *nblk = nwg;
    if (cg)
        hipLaunchKernelGGL((k_bj<N, T, true>), dim3(nwg), dim3(Cfg<N>::NT), 0, c->stream, r, z, S,
                           L, C, (int)c->n_cells, nwg, cg->x, cg->r, cg->p, cg->q, cg->sc,
                           c->cgpart, (int)c->n_cells + 1, (T)0, (T)0, 0, cg->pqp, cg->npq);
    else
        hipLaunchKernelGGL((k_bj<N, T, false>), dim3(nwg), dim3(Cfg<N>::NT), 0, c->stream, r, z, S,
                           L, C, (int)c->n_cells, nwg, (T *)nullptr, (T *)nullptr,
                           (const T *)nullptr, (const T *)nullptr, (const double *)nullptr,
                           (double *)nullptr, 0);
    return hipGetLastError();
}

template <typename T>
hipError_t bj_dispatch(hx_ctx *c, const T *r, T *z, const CgArgs<T> *cg = nullptr,
                       int *nblk = nullptr)
{
    switch (c->n) {
    case 2: return bj_n<2, T>(c, r, z, cg, nblk);
    case 3: return bj_n<3, T>(c, r, z, cg, nblk);
    case 4: return bj_n<4, T>(c, r, z, cg, nblk);
    case 5: return bj_n<5, T>(c, r, z, cg, nblk);
    case 6: return bj_n<6, T>(c, r, z, cg, nblk);
    case 7: return bj_n<7, T>(c, r, z, cg, nblk);
    case 8: return bj_n<8, T>(c, r, z, cg, nblk);
    default: return hipErrorInvalidValue;
    }
}

template <int N>
hipError_t bj_scaled_n(hx_ctx *c, const double *w, const double *part, int nb, double *v, double *z)
{
    const int cpb = Cfg<N>::CPB;
    const int nwg = (int)((c->n_cells + cpb - 1) / cpb);
    hipLaunchKernelGGL((k_bj<N, double, false>), dim3(nwg), dim3(Cfg<N>::NT), 0, c->stream, w, z,
                       c->bjS64, c->bjL64, c->bjC64, (int)c->n_cells, nwg, v, (double *)nullptr,
                       (const double *)nullptr, (const double *)nullptr, (const double *)nullptr,
                       const_cast<double *>(part), nb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_bj64(hx_ctx *c, const double *r, double *z) { return bj_dispatch<double>(c, r, z); }

hipError_t launch_bj64_scaled(hx_ctx *c, const double *w, const double *part, int nb, double *v,
                              double *z)
{
    if (nb < 1 || !part) return hipErrorInvalidValue;
    switch (c->n) {
    case 2: return bj_scaled_n<2>(c, w, part, nb, v, z);
    case 3: return bj_scaled_n<3>(c, w, part, nb, v, z);
    case 4: return bj_scaled_n<4>(c, w, part, nb, v, z);
    case 5: return bj_scaled_n<5>(c, w, part, nb, v, z);
    case 6: return bj_scaled_n<6>(c, w, part, nb, v, z);
    case 7: return bj_scaled_n<7>(c, w, part, nb, v, z);
    case 8: return bj_scaled_n<8>(c, w, part, nb, v, z);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bj_cheb64(hx_ctx *c, const double *r, double *d, double *x, double ca, double cb,
                            int read_d, int accum)
{
    return bj_cheb_dispatch<double>(c, r, d, x, ca, cb, read_d, accum);
}

hipError_t launch_bj_cheb32(hx_ctx *c, const float *r, float *d, float *x, double ca, double cb,
                            int read_d, int accum)
{
    return bj_cheb_dispatch<float>(c, r, d, x, ca, cb, read_d, accum);
}
hipError_t launch_bj32(hx_ctx *c, const float *r, float *z) { return bj_dispatch<float>(c, r, z); }

hipError_t launch_cg_bj64(hx_ctx *c, double *x, double *r, const double *p, const double *q,
                          double *z, const double *sc, int *nblk, const double *pqp, int npq)
{
    CgArgs<double> a;
    a.x = x; a.r = r; a.p = p; a.q = q; a.sc = sc; a.pqp = pqp; a.npq = npq;
    return bj_dispatch<double>(c, r, z, &a, nblk);
}

hipError_t launch_cg_bj32(hx_ctx *c, float *x, float *r, const float *p, const float *q, float *z,
                          const double *sc, int *nblk, const double *pqp, int npq)
{
    CgArgs<float> a;
    a.x = x; a.r = r; a.p = p; a.q = q; a.sc = sc; a.pqp = pqp; a.npq = npq;
    return bj_dispatch<float>(c, r, z, &a, nblk);
}

namespace {
// z = D^{-1} r with a stored inverse diagonal
template <typename T>
__global__ void k_diag(int64_t n, const T *__restrict__ dinv, const T *__restrict__ r, T *z)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) z[i] = dinv[i] * r[i];
}
}  // namespace

hipError_t launch_diag64(hx_ctx *c, int which, const double *r, double *z)
{
    const int64_t n = c->n_dofs;
    hipLaunchKernelGGL(k_diag<double>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n,
                       c->dg64 + (int64_t)which * n, r, z);
    return hipGetLastError();
}

hipError_t launch_diag32(hx_ctx *c, int which, const float *r, float *z)
{
    const int64_t n = c->n_dofs;
    hipLaunchKernelGGL(k_diag<float>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n,
                       c->dg32 + (int64_t)which * n, r, z);
    return hipGetLastError();
}

namespace {
// z = M^{-1} r for the alpha-weighted cell mass blocks
//   M_K = B3^T diag(m_K) B3,  B3 = B (x) B (x) B,
// B the square (k+1) x (k+1) interpolation from the nodes to the Gauss points
// and m_K the quadrature weights times alpha |det J| (component 0 of the
// merged cell data), so M_K^{-1} = B3^{-1} diag(1/m_K) B3^{-T}: the exact
// inverse by tensor-product sweeps (section 3.3, the inverse of the mass
// matrix as S^-T J^-1 S^-1 with S a Kronecker product of 1-D matrices), valid
// for curved cells and variable alpha.  Same thread mapping as k_bj, with the
// one 1-D matrix shared by all cells.
// FUSE: the conjugate-gradient step around it, as in k_bj.  With INV false
// the same sweeps apply M_K itself (B3^T diag(m_K) B3: the 1-D matrix is
// B^T, the scaling a product).  The weights are wgt[cell * wstride + q].
template <int N, typename T, bool FUSE, bool INV>
__global__ void __launch_bounds__(Cfg<N>::NT)
k_massinv(const T *__restrict__ rin, T *__restrict__ z, const T *__restrict__ wgt, int64_t wstride,
          const double *__restrict__ Fm, int n_cells, int nwg, T *x, T *rw,
          const T *__restrict__ p, const T *__restrict__ q, const double *__restrict__ sc,
          double *part, int ld, const double *__restrict__ pqp = nullptr, int npq = 0)
{
    const T *r = FUSE ? rw : rin;
    constexpr int NF = Cfg<N>::NF, ND = Cfg<N>::ND, CPB = Cfg<N>::CPB;
    __shared__ T sR[CPB][ND];
    __shared__ T sB[NF];                 // sB[i*N+q] = (B^{-1})_{iq}, or B_{qi}

    const int bid = blockIdx.x;
    const int q8 = nwg / NXCD, r8 = nwg % NXCD, xcd = bid % NXCD;
    const int wg = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / NXCD;
    const int t = threadIdx.x;
    const int lc0 = t / NF;
    const bool slot = lc0 < CPB;
    const int lc = slot ? lc0 : 0;
    const int tt = t - lc0 * NF;
    const int a = tt % N, b = tt / N;
    const int64_t cid = (int64_t)wg * CPB + lc;
    const bool active = slot && cid < n_cells;

    static_assert(NF <= Cfg<N>::NT, "one table entry per thread");
    const T fb = t < NF ? (T)(INV ? Fm[t] : Fm[(t % N) * N + t / N]) : T(0);
    T mq[N], v[N], w[N], rp[N];
    double acc_rr = 0.0, acc_rz = 0.0;
    double pq = 0.0;
    if (FUSE) {
        static_assert(!FUSE || Cfg<N>::NT == 256, "the fused step sums with a 256-thread workgroup");
        if (pqp) {
            __shared__ double shq[4];
            pq = sum256(pqp, npq, shq);
        } else {
            pq = sc[1];
        }
    }
    // every global load of the cell at once: the residual (and for the CG
    // step x, p and q) and the pencil's weights
    T rv[N], xv[N], pv[N], qv[N];
    if (active) {
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const int64_t gi = cid * ND + tt + u * NF;
            rv[u] = r[gi];
            if (FUSE) {
                xv[u] = x[gi];
                pv[u] = p[gi];
                qv[u] = q[gi];
            }
        }
#pragma unroll
        for (int m = 0; m < N; ++m) mq[m] = wgt[cid * wstride + a + N * b + NF * m];
    }
    __builtin_amdgcn_sched_barrier(0);
    if (t < NF) sB[t] = fb;
    if (FUSE && active) {
        const T al = (T)(pq != 0.0 ? sc[0] / pq : 0.0);
#pragma unroll
        for (int u = 0; u < N; ++u) {
            const int e = tt + u * NF;
            const int64_t gi = cid * ND + e;
            const T rn = rv[u] - al * qv[u];
            x[gi] = xv[u] + al * pv[u];
            rw[gi] = rn;
            sR[lc][e] = rn;
            acc_rr += (double)rn * (double)rn;
        }
    } else if (active) {
#pragma unroll
        for (int u = 0; u < N; ++u) sR[lc][tt + u * NF] = rv[u];
    }
    __syncthreads();
    // B^{-T} along x: thread (j=a, l=b); rp keeps the residual pencil, at the
    // positions of the output pencil written at the end
    if (active) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = rp[i] = sR[lc][i + N * a + NF * b];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            T s = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) s += sB[i * N + m] * v[i];
            w[m] = s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int m = 0; m < N; ++m) sR[lc][m + N * a + NF * b] = w[m];
    }
    __syncthreads();
    // B^{-T} along y: thread (qx=a, l=b)
    if (active) {
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = sR[lc][a + N * j + NF * b];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            T s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += sB[j * N + m] * v[j];
            w[m] = s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int m = 0; m < N; ++m) sR[lc][a + N * m + NF * b] = w[m];
    }
    __syncthreads();
    // B^{-T} along z, 1/m at the Gauss points, B^{-1} along z: thread (qx=a, qy=b);
    // the Gauss point (a, b, m) is entry a + N b + N^2 m of the cell data
    if (active) {
#pragma unroll
        for (int l = 0; l < N; ++l) v[l] = sR[lc][a + N * b + NF * l];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            T s = 0;
#pragma unroll
            for (int l = 0; l < N; ++l) s += sB[l * N + m] * v[l];
            w[m] = INV ? s / mq[m] : s * mq[m];
        }
#pragma unroll
        for (int l = 0; l < N; ++l) {
            T s = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) s += sB[l * N + m] * w[m];
            v[l] = s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int l = 0; l < N; ++l) sR[lc][a + N * b + NF * l] = v[l];
    }
    __syncthreads();
    // B^{-1} along y: thread (qx=a, l=b)
    if (active) {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = sR[lc][a + N * m + NF * b];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T s = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) s += sB[j * N + m] * v[m];
            w[j] = s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int j = 0; j < N; ++j) sR[lc][a + N * j + NF * b] = w[j];
    }
    __syncthreads();
    // B^{-1} along x: thread (j=a, l=b), output through LDS for contiguous stores
    if (active) {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = sR[lc][m + N * a + NF * b];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) s += sB[i * N + m] * v[m];
            w[i] = s;
            acc_rz += (double)rp[i] * (double)s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < N; ++i) sR[lc][i + N * a + NF * b] = w[i];
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int u = 0; u < N; ++u) z[cid * ND + tt + u * NF] = sR[lc][tt + u * NF];
    }
    if (FUSE) {
        __shared__ double sh2[2 * (Cfg<N>::NT / 64)];
        block_sum2<Cfg<N>::NT>(acc_rz, acc_rr, sh2);
        if (threadIdx.x == 0) {
            part[bid] = acc_rz;
            part[ld + bid] = acc_rr;
        }
    }
}

template <int N, typename T>
hipError_t massinv_n(hx_ctx *c, const T *wgt, int64_t wstride, bool inv, const T *r, T *z,
                     const CgArgs<T> *cg, int *nblk)
{
    const int cpb = Cfg<N>::CPB;
    const int nwg = (int)((c->n_cells + cpb - 1) / cpb);
    const char *ref = reinterpret_cast<const char *>(c->ref);
    const double *Fm = reinterpret_cast<const double *>(ref + (inv ? offsetof(RefTab64, Binv)
                                                                     : offsetof(RefTab64, B)));
    if (nblk) *nblk = nwg;
    if (cg)
        hipLaunchKernelGGL((k_massinv<N, T, true, true>), dim3(nwg), dim3(Cfg<N>::NT), 0, c->stream,
                           r, z, wgt, wstride, Fm, (int)c->n_cells, nwg, cg->x, cg->r, cg->p, cg->q,
                           cg->sc, c->cgpart, (int)c->n_cells + 1, cg->pqp, cg->npq);
    else if (inv)
        hipLaunchKernelGGL((k_massinv<N, T, false, true>), dim3(nwg), dim3(Cfg<N>::NT), 0, c->stream,
                           r, z, wgt, wstride, Fm, (int)c->n_cells, nwg, (T *)nullptr, (T *)nullptr,
                           (const T *)nullptr, (const T *)nullptr, (const double *)nullptr,
                           (double *)nullptr, 0);
    else
        hipLaunchKernelGGL((k_massinv<N, T, false, false>), dim3(nwg), dim3(Cfg<N>::NT), 0, c->stream,
                           r, z, wgt, wstride, Fm, (int)c->n_cells, nwg, (T *)nullptr, (T *)nullptr,
                           (const T *)nullptr, (const T *)nullptr, (const double *)nullptr,
                           (double *)nullptr, 0);
    return hipGetLastError();
}

// the alpha-weighted mass of the Helmholtz operator: first cell-data component
template <typename T>
hipError_t massinv_dispatch(hx_ctx *c, const T *r, T *z, const CgArgs<T> *cg = nullptr,
                            int *nblk = nullptr, const T *wgt = nullptr, int64_t wstride = 0,
                            bool inv = true)
{
    if (!wgt) {
        wgt = std::is_same<T, double>::value ? (const T *)c->cell64 : (const T *)c->cell32;
        wstride = 7 * (int64_t)c->nd;
    }
    switch (c->n) {
    case 2: return massinv_n<2, T>(c, wgt, wstride, inv, r, z, cg, nblk);
    case 3: return massinv_n<3, T>(c, wgt, wstride, inv, r, z, cg, nblk);
    case 4: return massinv_n<4, T>(c, wgt, wstride, inv, r, z, cg, nblk);
    case 5: return massinv_n<5, T>(c, wgt, wstride, inv, r, z, cg, nblk);
    case 6: return massinv_n<6, T>(c, wgt, wstride, inv, r, z, cg, nblk);
    case 7: return massinv_n<7, T>(c, wgt, wstride, inv, r, z, cg, nblk);
    case 8: return massinv_n<8, T>(c, wgt, wstride, inv, r, z, cg, nblk);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t launch_massinv64(hx_ctx *c, const double *r, double *z) { return massinv_dispatch<double>(c, r, z); }
hipError_t launch_massinv32(hx_ctx *c, const float *r, float *z) { return massinv_dispatch<float>(c, r, z); }

hipError_t launch_mass64(hx_ctx *c, const double *wgt, int64_t wstride, int inv, const double *r,
                         double *z)
{
    return massinv_dispatch<double>(c, r, z, nullptr, nullptr, wgt, wstride, inv != 0);
}

hipError_t launch_cg_massinv64(hx_ctx *c, double *x, double *r, const double *p, const double *q,
                               double *z, const double *sc, int *nblk, const double *pqp, int npq)
{
    CgArgs<double> a;
    a.x = x; a.r = r; a.p = p; a.q = q; a.sc = sc; a.pqp = pqp; a.npq = npq;
    return massinv_dispatch<double>(c, r, z, &a, nblk);
}

hipError_t launch_cg_massinv32(hx_ctx *c, float *x, float *r, const float *p, const float *q,
                               float *z, const double *sc, int *nblk, const double *pqp, int npq)
{
    CgArgs<float> a;
    a.x = x; a.r = r; a.p = p; a.q = q; a.sc = sc; a.pqp = pqp; a.npq = npq;
    return massinv_dispatch<float>(c, r, z, &a, nblk);
}

}  // namespace hx
