// Matrix-free action of the SIP-DG Helmholtz-type operator, cell integrals
// and face fluxes fused in one kernel (paper: section 2, Helmholtz equation
// for the pressure; section 3.1, mass plus dt-scaled enthalpy-weighted
// stiffness; section 3.3, tensor-product evaluation with (k+1) Gauss points).
//
// Layout and mapping on gfx950
//  * a workgroup handles CPB cells; each cell is served by N*N threads, one per
//    "pencil" of N values along one direction; the direction changes between
//    the sum-factorisation sweeps by staging the cell's values in LDS.
//  * the 1-D tables (GLL->GL interpolation B, derivative BD, end derivatives DL)
//    sit in constant memory; every loop over them is unrolled at compile time,
//    so their entries are wave-uniform scalar operands.
//  * cell data [cell][7][N^3] (m, G symmetric) and face data
//    [cell][3][7][N^2] (g-, g+, s of the +d face) are streamed once, coalesced.
//  * faces are evaluated cell-centrically: a cell computes, for each of its 6
//    faces, its own and its neighbour's value / reference-gradient traces at the
//    N^2 face Gauss points and accumulates the flux terms of its own test
//    functions only, so every output value is written by exactly one thread
//    (no atomics; results are bitwise reproducible).
//  * workgroups are remapped so that each XCD walks a contiguous range of
//    cells, which keeps the neighbours a cell reads in that XCD's L2.
#include "common.hpp"

#include <type_traits>

namespace hx {

__constant__ OpTab c_op[MAXN + 1];

hipError_t upload_op_tables_operator(const OpTab *all)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_op), all, sizeof(OpTab) * (MAXN + 1));
}

namespace {

template <typename T, int N>
__device__ __forceinline__ T tB(int q, int i)
{
    if constexpr (std::is_same<T, double>::value) return c_op[N].B[q * N + i];
    else return c_op[N].Bf[q * N + i];
}
template <typename T, int N>
__device__ __forceinline__ T tD(int q, int i)
{
    if constexpr (std::is_same<T, double>::value) return c_op[N].BD[q * N + i];
    else return c_op[N].BDf[q * N + i];
}
template <typename T, int N>
__device__ __forceinline__ T tE(int e, int i)
{
    if constexpr (std::is_same<T, double>::value) return c_op[N].DL[e][i];
    else return c_op[N].DLf[e][i];
}

template <int N>
struct Cfg {
    static constexpr int NF = N * N, ND = N * N * N;
    static constexpr int CPB = (256 / NF) > 0 ? 256 / NF : 1;
    static constexpr int NT = ((CPB * NF + 63) / 64) * 64;
};

// local index with coordinate m along direction d and (p, r) along the two
// other directions in increasing order
template <int N>
__device__ __forceinline__ int lix(int d, int m, int p, int r)
{
    return d == 0 ? m + N * (p + N * r) : (d == 1 ? p + N * (m + N * r) : p + N * (r + N * m));
}

template <int N, typename T>
__global__ void __launch_bounds__(Cfg<N>::NT)
k_apply(const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ bvec,
        const T *__restrict__ cell, const T *__restrict__ face, const int32_t *__restrict__ nbr,
        int n_cells, int nwg)
{
    constexpr int NF = Cfg<N>::NF, ND = Cfg<N>::ND, CPB = Cfg<N>::CPB;
    __shared__ T sU[CPB][ND];
    __shared__ T sV[CPB][ND];
    __shared__ T sW[3][CPB][ND];
    __shared__ T sF[CPB][10][NF];

    // contiguous cell ranges per XCD (workgroups are dealt round-robin to XCDs)
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

    if (active)
        for (int e = tt; e < ND; e += NF) sU[lc][e] = x[cid * ND + e];
    __syncthreads();

    T Y[N];
    // ------------------------------------------------------------ cell part
    {
        // x: thread (j=a, l=b) -> B u and BD u along x
        if (active) {
            T r[N];
#pragma unroll
            for (int i = 0; i < N; ++i) r[i] = sU[lc][i + N * a + NF * b];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                T s0 = 0, s1 = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    s0 += tB<T, N>(q, i) * r[i];
                    s1 += tD<T, N>(q, i) * r[i];
                }
                sW[0][lc][q + N * a + NF * b] = s0;
                sW[1][lc][q + N * a + NF * b] = s1;
            }
        }
        __syncthreads();
        // y: thread (qx=a, l=b)
        T c0[N], c1[N], c2[N];
        if (active) {
            T p0[N], p1[N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                p0[j] = sW[0][lc][a + N * j + NF * b];
                p1[j] = sW[1][lc][a + N * j + NF * b];
            }
#pragma unroll
            for (int q = 0; q < N; ++q) {
                T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
                for (int j = 0; j < N; ++j) {
                    s0 += tB<T, N>(q, j) * p0[j];
                    s1 += tD<T, N>(q, j) * p0[j];
                    s2 += tB<T, N>(q, j) * p1[j];
                }
                c0[q] = s0; c1[q] = s1; c2[q] = s2;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int q = 0; q < N; ++q) {
                sW[0][lc][a + N * q + NF * b] = c0[q];   // u (interpolated in x, y)
                sW[1][lc][a + N * q + NF * b] = c1[q];   // d/deta
                sW[2][lc][a + N * q + NF * b] = c2[q];   // d/dxi
            }
        }
        __syncthreads();
        // z: thread (qx=a, qy=b): values and reference gradient at the points,
        // quadrature-point operation, then the transposed z sweep
        T t0[N], t1[N], t2[N];
        if (active) {
            T p0[N], p1[N], p2[N];
#pragma unroll
            for (int l = 0; l < N; ++l) {
                p0[l] = sW[0][lc][a + N * b + NF * l];
                p1[l] = sW[1][lc][a + N * b + NF * l];
                p2[l] = sW[2][lc][a + N * b + NF * l];
            }
            T v[N], fx[N], fy[N], fz[N];
            const T *cd = cell + cid * 7 * ND + a + N * b;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                T u = 0, dz = 0, dy = 0, dx = 0;
#pragma unroll
                for (int l = 0; l < N; ++l) {
                    u += tB<T, N>(q, l) * p0[l];
                    dz += tD<T, N>(q, l) * p0[l];
                    dy += tB<T, N>(q, l) * p1[l];
                    dx += tB<T, N>(q, l) * p2[l];
                }
                const int o = NF * q;
                const T m = cd[o], gxx = cd[ND + o], gxy = cd[2 * ND + o], gxz = cd[3 * ND + o],
                        gyy = cd[4 * ND + o], gyz = cd[5 * ND + o], gzz = cd[6 * ND + o];
                v[q] = m * u;
                fx[q] = gxx * dx + gxy * dy + gxz * dz;
                fy[q] = gxy * dx + gyy * dy + gyz * dz;
                fz[q] = gxz * dx + gyz * dy + gzz * dz;
            }
#pragma unroll
            for (int l = 0; l < N; ++l) {
                T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    s0 += tB<T, N>(q, l) * v[q] + tD<T, N>(q, l) * fz[q];
                    s1 += tB<T, N>(q, l) * fy[q];
                    s2 += tB<T, N>(q, l) * fx[q];
                }
                t0[l] = s0; t1[l] = s1; t2[l] = s2;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int l = 0; l < N; ++l) {
                sW[0][lc][a + N * b + NF * l] = t0[l];
                sW[1][lc][a + N * b + NF * l] = t1[l];
                sW[2][lc][a + N * b + NF * l] = t2[l];
            }
        }
        __syncthreads();
        // y transposed: thread (qx=a, l=b)
        T s0v[N], s1v[N];
        if (active) {
            T p0[N], p1[N], p2[N];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                p0[q] = sW[0][lc][a + N * q + NF * b];
                p1[q] = sW[1][lc][a + N * q + NF * b];
                p2[q] = sW[2][lc][a + N * q + NF * b];
            }
#pragma unroll
            for (int j = 0; j < N; ++j) {
                T s0 = 0, s1 = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    s0 += tB<T, N>(q, j) * p0[q] + tD<T, N>(q, j) * p1[q];
                    s1 += tB<T, N>(q, j) * p2[q];
                }
                s0v[j] = s0; s1v[j] = s1;
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int j = 0; j < N; ++j) {
                sW[0][lc][a + N * j + NF * b] = s0v[j];
                sW[1][lc][a + N * j + NF * b] = s1v[j];
            }
        }
        __syncthreads();
        // x transposed: thread (j=a, l=b) owns the output pencil Y
        if (active) {
            T p0[N], p1[N];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                p0[q] = sW[0][lc][q + N * a + NF * b];
                p1[q] = sW[1][lc][q + N * a + NF * b];
            }
#pragma unroll
            for (int i = 0; i < N; ++i) {
                T s = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) s += tB<T, N>(q, i) * p0[q] + tD<T, N>(q, i) * p1[q];
                Y[i] = s;
            }
        }
        __syncthreads();
        // sW[0] becomes the accumulator of the y- and z-face terms
        if (active) {
#pragma unroll
            for (int i = 0; i < N; ++i) sW[0][lc][i + N * a + NF * b] = 0;
        }
    }

    // ------------------------------------------------------------ faces
    T *YF = &sW[0][lc][0];
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
#pragma unroll 1
        for (int s = 0; s < 2; ++s) {
            const int32_t nb = active ? nbr[cid * 6 + 2 * d + s] : -1;
            const bool fact = nb >= 0;
            const int eo = s, en = 1 - s;               // own / neighbour end along d
            __syncthreads();                            // previous face done with sV, sF, YF
            if (fact)
                for (int e = tt; e < ND; e += NF) sV[lc][e] = x[(int64_t)nb * ND + e];
            __syncthreads();
            // T1: thread (p=a, r=b): layer values and normal derivatives
            if (fact) {
                T lo = 0, dno = 0, ln = 0, dnn = 0;
#pragma unroll
                for (int m = 0; m < N; ++m) {
                    const int id = lix<N>(d, m, a, b);
                    const T uo = sU[lc][id], un = sV[lc][id];
                    dno += tE<T, N>(eo, m) * uo;
                    dnn += tE<T, N>(en, m) * un;
                    if (m == (eo ? N - 1 : 0)) lo = uo;
                    if (m == (en ? N - 1 : 0)) ln = un;
                }
                sF[lc][0][a + N * b] = lo;
                sF[lc][1][a + N * b] = dno;
                sF[lc][2][a + N * b] = ln;
                sF[lc][3][a + N * b] = dnn;
            }
            __syncthreads();
            // T2: thread (q1=a, r=b): interpolate along the first tangential direction
            if (fact) {
                T g[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int p = 0; p < N; ++p) {
                    const T f0o = sF[lc][0][p + N * b], f1o = sF[lc][1][p + N * b];
                    const T f0n = sF[lc][2][p + N * b], f1n = sF[lc][3][p + N * b];
                    const T bb = tB<T, N>(a, p), bd = tD<T, N>(a, p);
                    g[0] += bb * f0o; g[1] += bd * f0o; g[2] += bb * f1o;
                    g[3] += bb * f0n; g[4] += bd * f0n; g[5] += bb * f1n;
                }
#pragma unroll
                for (int k = 0; k < 6; ++k) sF[lc][4 + k][a + N * b] = g[k];
            }
            __syncthreads();
            // T3: thread (q1=a, q2=b): traces at the face point, flux terms
            if (fact) {
                T vo = 0, t2o = 0, t1o = 0, dno = 0, vn = 0, t2n = 0, t1n = 0, dnn = 0;
#pragma unroll
                for (int r = 0; r < N; ++r) {
                    const T bb = tB<T, N>(b, r), bd = tD<T, N>(b, r);
                    const T g0o = sF[lc][4][a + N * r], g1o = sF[lc][5][a + N * r], g2o = sF[lc][6][a + N * r];
                    const T g0n = sF[lc][7][a + N * r], g1n = sF[lc][8][a + N * r], g2n = sF[lc][9][a + N * r];
                    vo += bb * g0o; t2o += bd * g0o; t1o += bb * g1o; dno += bb * g2o;
                    vn += bb * g0n; t2n += bd * g0n; t1n += bb * g1n; dnn += bb * g2n;
                }
                const int64_t fid = s ? cid : (int64_t)nb;
                const T *fd = face + (fid * 3 + d) * 7 * NF + a + N * b;
                const T gm0 = fd[0], gm1 = fd[NF], gm2 = fd[2 * NF];
                const T gp0 = fd[3 * NF], gp1 = fd[4 * NF], gp2 = fd[5 * NF];
                const T pen = fd[6 * NF];
                // reference gradients in (xi, eta, zeta) order
                T go[3], gn[3];
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                go[d] = dno; go[t1] = t1o; go[t2] = t2o;
                gn[d] = dnn; gn[t1] = t1n; gn[t2] = t2n;
                const T fo = s ? (gm0 * go[0] + gm1 * go[1] + gm2 * go[2])
                               : (gp0 * go[0] + gp1 * go[1] + gp2 * go[2]);
                const T fn = s ? (gp0 * gn[0] + gp1 * gn[1] + gp2 * gn[2])
                               : (gm0 * gn[0] + gm1 * gn[1] + gm2 * gn[2]);
                const T flux = fo + fn;
                const T jump = s ? (vo - vn) : (vn - vo);
                const T sg = s ? T(1) : T(-1);
                const T cv = sg * (T(-0.5) * flux + pen * jump);
                const T hj = T(-0.5) * jump;
                T cg[3];
                cg[0] = hj * (s ? gm0 : gp0);
                cg[1] = hj * (s ? gm1 : gp1);
                cg[2] = hj * (s ? gm2 : gp2);
                sF[lc][0][a + N * b] = cv;
                sF[lc][1][a + N * b] = cg[t2];
                sF[lc][2][a + N * b] = cg[t1];
                sF[lc][3][a + N * b] = cg[d];
            }
            __syncthreads();
            // R2: thread (q1=a, r=b): transpose along the second tangential direction
            if (fact) {
                T h0 = 0, h1 = 0, h2 = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    const T bb = tB<T, N>(q, b), bd = tD<T, N>(q, b);
                    h0 += bb * sF[lc][0][a + N * q] + bd * sF[lc][1][a + N * q];
                    h1 += bb * sF[lc][2][a + N * q];
                    h2 += bb * sF[lc][3][a + N * q];
                }
                sF[lc][4][a + N * b] = h0;
                sF[lc][5][a + N * b] = h1;
                sF[lc][6][a + N * b] = h2;
            }
            __syncthreads();
            // R1 + R0: thread (p=a, r=b): transpose along the first tangential
            // direction, then spread onto the own normal pencil
            if (fact) {
                T f0 = 0, f1 = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    const T bb = tB<T, N>(q, a), bd = tD<T, N>(q, a);
                    f0 += bb * sF[lc][4][q + N * b] + bd * sF[lc][5][q + N * b];
                    f1 += bb * sF[lc][6][q + N * b];
                }
                if (d == 0) {
#pragma unroll
                    for (int m = 0; m < N; ++m)
                        Y[m] += tE<T, N>(eo, m) * f1 + ((m == (eo ? N - 1 : 0)) ? f0 : T(0));
                } else {
#pragma unroll
                    for (int m = 0; m < N; ++m) {
                        const int id = lix<N>(d, m, a, b);
                        YF[id] += tE<T, N>(eo, m) * f1 + ((m == (eo ? N - 1 : 0)) ? f0 : T(0));
                    }
                }
            }
        }
    }
    __syncthreads();
    if (active) {
        const int64_t o = cid * ND + N * a + NF * b;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const T val = Y[i] + YF[i + N * a + NF * b];
            y[o + i] = bvec ? bvec[o + i] - val : val;
        }
    }
}

template <int N, typename T>
hipError_t apply_n(hx_ctx *c, const T *x, T *y, const T *b)
{
    const int cpb = Cfg<N>::CPB;
    const int nwg = (int)((c->n_cells + cpb - 1) / cpb);
    const T *cell = std::is_same<T, double>::value ? (const T *)c->cell64 : (const T *)c->cell32;
    const T *face = std::is_same<T, double>::value ? (const T *)c->face64 : (const T *)c->face32;
    hipLaunchKernelGGL((k_apply<N, T>), dim3(nwg), dim3(Cfg<N>::NT), 0, c->stream, x, y, b, cell,
                       face, c->nbr, (int)c->n_cells, nwg);
    return hipGetLastError();
}

template <typename T>
hipError_t apply_dispatch(hx_ctx *c, const T *x, T *y, const T *b)
{
    switch (c->n) {
    case 2: return apply_n<2, T>(c, x, y, b);
    case 3: return apply_n<3, T>(c, x, y, b);
    case 4: return apply_n<4, T>(c, x, y, b);
    case 5: return apply_n<5, T>(c, x, y, b);
    case 6: return apply_n<6, T>(c, x, y, b);
    case 7: return apply_n<7, T>(c, x, y, b);
    case 8: return apply_n<8, T>(c, x, y, b);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_apply64(hx_ctx *c, const double *x, double *y, const double *b)
{
    return apply_dispatch<double>(c, x, y, b);
}

hipError_t launch_apply32(hx_ctx *c, const float *x, float *y, const float *b)
{
    return apply_dispatch<float>(c, x, y, b);
}

}  // namespace hx
