// Non-conforming (2:1) faces: a face of a coarse cell split into four
// quarters, each the whole face of a fine cell (the paper's second mesh
// refines part of its domain, section 3).  Every quarter carries the same
// interior-penalty terms as a conforming face, integrated with the fine
// face's (k+1)^2 Gauss points; the coarse side is evaluated at the images of
// those points on its face, ((s1 + xi_1)/2, (s2 + xi_2)/2) for quarter
// s = s1 + 2 s2; ds and the unit normal n (the +d direction, the minus cell's
// outward normal) come from the fine side; the minus cell is the one whose
// +d face it is; sigma = P (k+1)^2 max(|S|/|K_fine|, |S|/|K_coarse|).
//
// The operator kernel treats these faces as absent (neighbour -2); after it,
// k_hang_apply computes each quarter's contributions to the test functions
// of both cells (one workgroup per quarter, no atomics) into a staging
// buffer, and k_hang_gather adds them to y cell by cell in a fixed order, so
// results stay bitwise reproducible.  The set-up kernels evaluate the basis
// and the map at the points directly (Lagrange evaluation); the apply kernel
// sum-factorises on the face.
//
// Records: {C, fc, F, s}: face fc (0..5 = -x, +x, -y, +y, -z, +z) of the
// coarse cell C, face fc ^ 1 of the fine cell F, quarter s.  Point (a, b) of
// a quarter is stored at a + n b, a along the first and b along the second
// tangential direction.
#include "common.hpp"

namespace hx {
namespace {

// Lagrange basis through the n nodes xl: values and derivatives at t
template <typename R>
__device__ inline void lag_nodes(int n, const double *xl, double t, R *v, R *d)
{
    for (int i = 0; i < n; ++i) {
        double val = 1.0, der = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == i) continue;
            const double f = (t - xl[m]) / (xl[i] - xl[m]);
            der = der * f + val / (xl[i] - xl[m]);
            val *= f;
        }
        v[i] = (R)val;
        d[i] = (R)der;
    }
}

// Lagrange basis through the equispaced geometry nodes a/g
__device__ inline void lag_equi_h(int ng, double t, double *v, double *d)
{
    const double g = ng - 1;
    for (int i = 0; i < ng; ++i) {
        const double xi = i / g;
        double val = 1.0, der = 0.0;
        for (int m = 0; m < ng; ++m) {
            if (m == i) continue;
            const double xm = m / g;
            const double f = (t - xm) / (xi - xm);
            der = der * f + val / (xi - xm);
            val *= f;
        }
        v[i] = val;
        d[i] = der;
    }
}

__device__ inline void map_jac(const double *__restrict__ X, int ng, const double xi[3], double J[3][3])
{
    double v[3][MAXG + 1], d[3][MAXG + 1];
    for (int c = 0; c < 3; ++c) lag_equi_h(ng, xi[c], v[c], d[c]);
    for (int r = 0; r < 3; ++r) J[r][0] = J[r][1] = J[r][2] = 0.0;
    for (int cz = 0; cz < ng; ++cz)
        for (int cy = 0; cy < ng; ++cy)
            for (int cx = 0; cx < ng; ++cx) {
                const double *P = X + 3 * (cx + ng * (cy + ng * cz));
                const double s0 = d[0][cx] * v[1][cy] * v[2][cz], s1 = v[0][cx] * d[1][cy] * v[2][cz],
                             s2 = v[0][cx] * v[1][cy] * d[2][cz];
                for (int r = 0; r < 3; ++r) {
                    J[r][0] += s0 * P[r];
                    J[r][1] += s1 * P[r];
                    J[r][2] += s2 * P[r];
                }
            }
}

__device__ inline void inv3h(const double J[3][3], double Ji[3][3], double *det)
{
    const double dt = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                      J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    const double id = 1.0 / dt;
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    *det = dt;
}

// reference points of quarter point (a, b) on the fine (xiF) and coarse (xiC)
// cell
__device__ inline void quarter_points(const RefTab64 *T, const int32_t *h, int a, int b, double xiF[3],
                                      double xiC[3])
{
    const int fc = h[1], d = fc >> 1, s = h[3];
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    xiF[d] = ((fc ^ 1) & 1) ? 1.0 : 0.0;
    xiF[t1] = T->xq[a];
    xiF[t2] = T->xq[b];
    xiC[d] = (fc & 1) ? 1.0 : 0.0;
    xiC[t1] = 0.5 * ((s & 1) + T->xq[a]);
    xiC[t2] = 0.5 * ((s >> 1) + T->xq[b]);
}

// geometric factors (thread per quarter point): [h][7][nf] =
// ds J_C^-1 n (3, coarse reference axes), ds J_F^-1 n (3, fine axes), ds/2
__global__ void k_hang_geom(const double *__restrict__ nodes, int ng, int n, int64_t n_hang,
                            const int32_t *__restrict__ hang, const RefTab64 *__restrict__ T,
                            double *hgeo)
{
    const int nf = n * n;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_hang * nf) return;
    const int64_t h = t / nf;
    const int pt = (int)(t % nf), a = pt % n, b = pt / n;
    const int32_t *rec = hang + 4 * h;
    const int d = rec[1] >> 1;
    double xiF[3], xiC[3], J[3][3], JiF[3][3], JiC[3][3], detF, detC;
    quarter_points(T, rec, a, b, xiF, xiC);
    const int64_t gsz = (int64_t)ng * ng * ng * 3;
    map_jac(nodes + rec[2] * gsz, ng, xiF, J);
    inv3h(J, JiF, &detF);
    map_jac(nodes + rec[0] * gsz, ng, xiC, J);
    inv3h(J, JiC, &detC);
    // n = J_F^-T e_d / |J_F^-T e_d|: row d of J_F^-1
    double nv[3] = {JiF[d][0], JiF[d][1], JiF[d][2]};
    const double len = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    for (int r = 0; r < 3; ++r) nv[r] /= len;
    const double ds = T->wq[a] * T->wq[b] * detF * len;
    double *g = hgeo + h * 7 * nf + pt;
    for (int r = 0; r < 3; ++r) {
        g[r * nf] = ds * (JiC[r][0] * nv[0] + JiC[r][1] * nv[1] + JiC[r][2] * nv[2]);
        g[(3 + r) * nf] = ds * (JiF[r][0] * nv[0] + JiF[r][1] * nv[1] + JiF[r][2] * nv[2]);
    }
    g[6 * nf] = 0.5 * ds;
}

// area and penalty of each quarter (thread per quarter)
__global__ void k_hang_sigma(int n, int64_t n_hang, const int32_t *__restrict__ hang,
                             const double *__restrict__ hgeo, const double *__restrict__ vol, double P,
                             double *hsig, double *harea)
{
    const int nf = n * n;
    const int64_t h = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (h >= n_hang) return;
    double area = 0.0;
    for (int pt = 0; pt < nf; ++pt) area += 2.0 * hgeo[h * 7 * nf + 6 * nf + pt];
    const int32_t *rec = hang + 4 * h;
    const double r = fmax(area / vol[rec[2]], area / vol[rec[0]]);
    hsig[h] = P * (double)nf * r;
    harea[h] = area;
}

// merged data (thread per quarter point): gC = beta_C ds J_C^-1 n,
// gF = beta_F ds J_F^-1 n, s = sigma (beta_C + beta_F) ds / 2
__global__ void k_hang_coef(int n, int64_t n_hang, const int32_t *__restrict__ hang,
                            const RefTab64 *__restrict__ T, const double *__restrict__ beta,
                            const double *__restrict__ hgeo, const double *__restrict__ hsig,
                            double *hd64, float *hd32)
{
    const int nf = n * n, nd = nf * n;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n_hang * nf) return;
    const int64_t h = t / nf;
    const int pt = (int)(t % nf), a = pt % n, b = pt / n;
    const int32_t *rec = hang + 4 * h;
    double xi[2][3];
    quarter_points(T, rec, a, b, xi[1], xi[0]);
    double bv[2];
    for (int side = 0; side < 2; ++side) {
        double v[3][MAXN], dd[3][MAXN];
        for (int c = 0; c < 3; ++c) lag_nodes<double>(n, T->xl, xi[side][c], v[c], dd[c]);
        const double *bc = beta + (int64_t)(side ? rec[2] : rec[0]) * nd;
        double s = 0.0;
        for (int l = 0; l < n; ++l)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) s += v[0][i] * v[1][j] * v[2][l] * bc[i + n * (j + n * l)];
        bv[side] = s;
    }
    const double *g = hgeo + h * 7 * nf + pt;
    double out[7];
    for (int r = 0; r < 3; ++r) {
        out[r] = bv[0] * g[r * nf];
        out[3 + r] = bv[1] * g[(3 + r) * nf];
    }
    out[6] = hsig[h] * (bv[0] + bv[1]) * g[6 * nf];
    for (int s = 0; s < 7; ++s) {
        hd64[h * 7 * nf + s * nf + pt] = out[s];
        hd32[h * 7 * nf + s * nf + pt] = (float)out[s];
    }
}

// contributions of one quarter to the test functions of both cells (one
// wave per quarter): contrib[h][side][nd], side 0 coarse, 1 fine.  Both
// sides' traces are sum-factorised on the face: items (side, i1, i2) take the
// face layer and the normal-derivative column (GLL nodes lie on the face, so
// the normal direction needs the end node and the derivative weights only),
// items (side, a, i2) contract along the first tangential direction with the
// side's 1-D tables at the quarter's points (the coarse side's at
// ((s + xi)/2)), items (a, b) along the second and form the flux terms of
// both sides, and the same steps run backwards to the face layer and the
// normal lines, which each item (side, i1, i2) writes whole.
template <int N, typename T>
__global__ void __launch_bounds__(64)
k_hang_apply(int64_t n_hang, const int32_t *__restrict__ hang, const RefTab64 *__restrict__ TB,
             const T *__restrict__ hd, const T *__restrict__ x, T *__restrict__ contrib)
{
    constexpr int NF = N * N, ND = NF * N;
    __shared__ T tb[2][2][2][NF];          // [side][tangential axis][value, derivative][a * N + i]
    __shared__ T sDL[2][N];                // l_m'(0), l_m'(1)
    __shared__ T Lv[2][NF], Ld[2][NF];     // face layer and normal derivative, [side][i1 + N i2]
    __shared__ T T0[2][NF], T1[2][NF], T2[2][NF];   // along t1, [side][a + N i2]
    __shared__ T Wv[2][NF], Wa[2][NF], Wb[2][NF], Wn[2][NF];   // weights per point a + N b
    __shared__ T Gv[2][NF], Gb[2][NF], Gn[2][NF];   // back along t1, [side][i1 + N b]
    const int64_t h = blockIdx.x;
    const int32_t *rec = hang + 4 * h;
    const int fc = rec[1], d = fc >> 1, sq = rec[3];
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int st[3] = {1, N, NF};
    const int s1 = st[t1], s2 = st[t2], sn = st[d];
    // end node along the normal: the coarse cell's face fc, the fine cell's fc ^ 1
    const int eside[2] = {(fc & 1) ? 1 : 0, ((fc ^ 1) & 1) ? 1 : 0};
    const int minus = (fc & 1) ? 0 : 1;
    const T *xs[2] = {x + (int64_t)rec[0] * ND, x + (int64_t)rec[2] * ND};
    const int tid = threadIdx.x;
    // 1-D tables: fine side from the set-up tables, coarse side at the
    // quarter's points
    if (tid < 2 * N) {
        const int ax = tid / N, a = tid % N;
        const int half = ax == 0 ? (sq & 1) : (sq >> 1);
        T v[N], dv[N];
        lag_nodes<T>(N, TB->xl, 0.5 * (half + TB->xq[a]), v, dv);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            tb[0][ax][0][a * N + i] = v[i];
            tb[0][ax][1][a * N + i] = dv[i];
        }
    }
    for (int e = tid; e < 2 * NF; e += 64) {
        const int ax = e / NF, k = e % NF;
        tb[1][ax][0][k] = (T)TB->B[k];
        tb[1][ax][1][k] = (T)TB->BD[k];
    }
    if (tid < 2 * N) sDL[tid / N][tid % N] = (T)TB->DL[tid / N][tid % N];
    __syncthreads();
    // face layer and normal derivative: item (side, i1, i2)
    for (int it = tid; it < 2 * NF; it += 64) {
        const int side = it / NF, k = it % NF;
        const int i1 = k % N, i2 = k / N;
        const T *xp = xs[side] + i1 * s1 + i2 * s2;
        const int e = eside[side];
        T dn = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) dn += sDL[e][m] * xp[m * sn];
        Lv[side][k] = xp[(e ? N - 1 : 0) * sn];
        Ld[side][k] = dn;
    }
    __syncthreads();
    // along t1: item (side, a, i2)
    for (int it = tid; it < 2 * NF; it += 64) {
        const int side = it / NF, k = it % NF;
        const int a = k % N, i2 = k / N;
        const T *B1 = tb[side][0][0] + a * N, *D1 = tb[side][0][1] + a * N;
        T c0 = 0, c1 = 0, c2 = 0;
#pragma unroll
        for (int i1 = 0; i1 < N; ++i1) {
            c0 += B1[i1] * Lv[side][i1 + N * i2];
            c1 += D1[i1] * Lv[side][i1 + N * i2];
            c2 += B1[i1] * Ld[side][i1 + N * i2];
        }
        T0[side][k] = c0;
        T1[side][k] = c1;
        T2[side][k] = c2;
    }
    __syncthreads();
    // along t2 and the flux terms at point (a, b): both sides in one item
    for (int pt = tid; pt < NF; pt += 64) {
        const int a = pt % N, b = pt / N;
        T u[2], gr[2][3];
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const T *B2 = tb[sd][1][0] + b * N, *D2 = tb[sd][1][1] + b * N;
            T v = 0, ga = 0, gb = 0, gn = 0;
#pragma unroll
            for (int i2 = 0; i2 < N; ++i2) {
                v += B2[i2] * T0[sd][a + N * i2];
                ga += B2[i2] * T1[sd][a + N * i2];
                gb += D2[i2] * T0[sd][a + N * i2];
                gn += B2[i2] * T2[sd][a + N * i2];
            }
            u[sd] = v;
            gr[sd][t1] = ga;
            gr[sd][t2] = gb;
            gr[sd][d] = gn;
        }
        const T *g = hd + h * 7 * NF + pt;
        T flux = 0;
#pragma unroll
        for (int r = 0; r < 3; ++r) flux += g[r * NF] * gr[0][r] + g[(3 + r) * NF] * gr[1][r];
        const T jump = u[minus] - u[1 - minus];
        const T pen = g[6 * NF];
#pragma unroll
        for (int sd = 0; sd < 2; ++sd) {
            const T z = sd == minus ? T(1) : T(-1);
            const T hj = T(-0.5) * jump;
            Wv[sd][pt] = z * (T(-0.5) * flux + pen * jump);
            Wa[sd][pt] = hj * g[(3 * sd + t1) * NF];
            Wb[sd][pt] = hj * g[(3 * sd + t2) * NF];
            Wn[sd][pt] = hj * g[(3 * sd + d) * NF];
        }
    }
    __syncthreads();
    // back along t1: item (side, i1, b)
    for (int it = tid; it < 2 * NF; it += 64) {
        const int side = it / NF, k = it % NF;
        const int i1 = k % N, b = k / N;
        const T *B1 = tb[side][0][0], *D1 = tb[side][0][1];
        T gv = 0, gb = 0, gn = 0;
#pragma unroll
        for (int a = 0; a < N; ++a) {
            const int pt = a + N * b;
            gv += B1[a * N + i1] * Wv[side][pt] + D1[a * N + i1] * Wa[side][pt];
            gb += B1[a * N + i1] * Wb[side][pt];
            gn += B1[a * N + i1] * Wn[side][pt];
        }
        Gv[side][k] = gv;
        Gb[side][k] = gb;
        Gn[side][k] = gn;
    }
    __syncthreads();
    // back along t2 and out: item (side, i1, i2) writes its normal line
    for (int it = tid; it < 2 * NF; it += 64) {
        const int side = it / NF, k = it % NF;
        const int i1 = k % N, i2 = k / N;
        const T *B2 = tb[side][1][0], *D2 = tb[side][1][1];
        T f0 = 0, f1 = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) {
            f0 += B2[b * N + i2] * Gv[side][i1 + N * b] + D2[b * N + i2] * Gb[side][i1 + N * b];
            f1 += B2[b * N + i2] * Gn[side][i1 + N * b];
        }
        const int e = eside[side];
        T *out = contrib + (h * 2 + side) * ND + i1 * s1 + i2 * s2;
#pragma unroll
        for (int m = 0; m < N; ++m) out[m * sn] = sDL[e][m] * f1 + (m == (e ? N - 1 : 0) ? f0 : T(0));
    }
}

// y[cell] += (or -=, residual form) the staged contributions of its quarters,
// in the fixed order of its list (block per listed cell)
template <typename T>
__global__ void k_hang_gather(int nd, const int32_t *__restrict__ cells, const int32_t *__restrict__ ptr,
                              const int32_t *__restrict__ list, const T *__restrict__ contrib, T *y,
                              T sign)
{
    const int64_t k = blockIdx.x;
    const int64_t cell = cells[k];
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
        T s = 0;
        for (int e = ptr[k]; e < ptr[k + 1]; ++e) s += contrib[(int64_t)list[e] * nd + i];
        y[cell * nd + i] += sign * s;
    }
}

template <int N, typename T>
hipError_t hang_apply_n(hx_ctx *c, const T *x, T *y, bool residual)
{
    const bool f64 = sizeof(T) == 8;
    T *contrib = f64 ? (T *)c->hcontrib64 : (T *)c->hcontrib32;
    const T *hd = f64 ? (const T *)c->hdata64 : (const T *)c->hdata32;
    hipLaunchKernelGGL((k_hang_apply<N, T>), dim3((unsigned)c->n_hang), dim3(64), 0, c->stream, c->n_hang,
                       c->hang, c->ref, hd, x, contrib);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_hang_gather<T>), dim3((unsigned)c->n_hcell), dim3(128), 0, c->stream, c->nd,
                       c->hcells, c->hptr, c->hlist, (const T *)contrib, y, residual ? T(-1) : T(1));
    return hipGetLastError();
}

template <typename T>
hipError_t hang_dispatch(hx_ctx *c, const T *x, T *y, bool residual)
{
    switch (c->n) {
    case 2: return hang_apply_n<2, T>(c, x, y, residual);
    case 3: return hang_apply_n<3, T>(c, x, y, residual);
    case 4: return hang_apply_n<4, T>(c, x, y, residual);
    case 5: return hang_apply_n<5, T>(c, x, y, residual);
    case 6: return hang_apply_n<6, T>(c, x, y, residual);
    case 7: return hang_apply_n<7, T>(c, x, y, residual);
    case 8: return hang_apply_n<8, T>(c, x, y, residual);
    default: return hipErrorInvalidValue;
    }
}

inline unsigned nblk_h(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

hipError_t launch_hang_geometry(hx_ctx *c)
{
    const int64_t nt = c->n_hang * c->nf;
    hipLaunchKernelGGL(k_hang_geom, dim3(nblk_h(nt, 64)), dim3(64), 0, c->stream, c->nodes, c->g + 1, c->n,
                       c->n_hang, c->hang, c->ref, c->hgeo);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hang_sigma, dim3(nblk_h(c->n_hang, 64)), dim3(64), 0, c->stream, c->n, c->n_hang,
                       c->hang, c->hgeo, c->vol, c->P, c->hsig, c->harea);
    return hipGetLastError();
}

hipError_t launch_hang_coefficients(hx_ctx *c, const double *beta)
{
    const int64_t nt = c->n_hang * c->nf;
    hipLaunchKernelGGL(k_hang_coef, dim3(nblk_h(nt, 64)), dim3(64), 0, c->stream, c->n, c->n_hang, c->hang,
                       c->ref, beta, c->hgeo, c->hsig, c->hdata64, c->hdata32);
    return hipGetLastError();
}

hipError_t launch_hang_apply64(hx_ctx *c, const double *x, double *y, bool residual)
{
    return hang_dispatch<double>(c, x, y, residual);
}

hipError_t launch_hang_apply32(hx_ctx *c, const float *x, float *y, bool residual)
{
    return hang_dispatch<float>(c, x, y, residual);
}

}  // namespace hx
