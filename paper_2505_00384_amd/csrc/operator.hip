// Matrix-free action of the SIP-DG Helmholtz-type operator, cell integrals
// and face fluxes fused in one kernel (paper: section 2, Helmholtz equation
// for the pressure; section 3.1, mass plus dt-scaled enthalpy-weighted
// stiffness; section 3.3, tensor-product evaluation with (k+1) Gauss points).
//
// Layout and mapping on gfx950
//  * a workgroup is one wave64; it serves CPW cells with LPC lanes each
//    (N = 5: 2 cells x 32 lanes), so every barrier is a single-wave barrier.
//  * cell integrals: lane (a, b) owns a pencil of N values; the sweeps
//    (GLL -> Gauss interpolation B, derivative BD, and their transposes) run in
//    registers, and the pencil direction changes through LDS;
//  * face integrals: lane (f, p) owns column p of face f (6 faces x N
//    columns).  It reads the neighbour's normal lines straight from global
//    memory into registers at the start (in the same round trip as the own
//    values; the N lanes of a face read neighbouring addresses) and the own
//    ones from LDS, forms layer values and normal derivatives and interpolates
//    along the second tangential direction in registers; after one LDS
//    transpose lane (f, q2) finishes the first direction, the pointwise flux
//    terms at the Gauss points (face data laid out [comp][q1][q2], so these
//    loads are contiguous across lanes too) and the transposed sweep; a second
//    transpose returns to columns for the last transposed sweep.  The
//    pencil owners then add the six faces' layer and normal-derivative
//    contributions to their own output values.  Each output value is written
//    by exactly one lane (no atomics; bitwise reproducible).
//  * the 1-D tables sit in constant memory, loops over them are unrolled, so
//    their entries are wave-uniform scalar operands.
//  * cell data [cell][7][N^3] is streamed once with non-temporal loads; x and
//    the face data [cell][3][7][N][N] are read by neighbours too and stay
//    cacheable.
//  * cells are visited in the order of a host-built permutation: tiles of
//    columns swept layer by layer, in one contiguous range per XCD, so the
//    neighbours a cell reads were touched recently by the same XCD's L2.
#include "common.hpp"

#include <type_traits>

namespace hx {

__constant__ OpTab c_op[MAXN + 1];

hipError_t upload_op_tables_operator(const OpTab *all)
{
    return hipMemcpyToSymbol(HIP_SYMBOL(c_op), all, sizeof(OpTab) * (MAXN + 1));
}

namespace {

// compile-time copies of the same tables (generated at build time from the
// library's rules): with every loop unrolled the compiler materialises the
// entries with scalar moves instead of constant-memory loads
template <int N> struct KB;
template <int N> struct KBD;
template <int N> struct KDL;
#include "optables.inc"

template <typename T, int N>
__device__ __forceinline__ T tB(int q, int i)
{
    if constexpr (std::is_same<T, double>::value) return KB<N>::d[q * N + i];
    else return KB<N>::f[q * N + i];
}
template <typename T, int N>
__device__ __forceinline__ T tD(int q, int i)
{
    if constexpr (std::is_same<T, double>::value) return KBD<N>::d[q * N + i];
    else return KBD<N>::f[q * N + i];
}
template <typename T, int N>
__device__ __forceinline__ T tE(int e, int i)
{
    if constexpr (std::is_same<T, double>::value) return KDL<N>::d[e * N + i];
    else return KDL<N>::f[e * N + i];
}

constexpr int pow2_at_least(int v)
{
    int p = 1;
    while (p < v) p *= 2;
    return p;
}

template <int N>
struct Cfg {
    static constexpr int NF = N * N, ND = N * N * N;
    static constexpr int LPC = pow2_at_least(NF > 6 * N ? NF : 6 * N) > 64
                                   ? 64 : pow2_at_least(NF > 6 * N ? NF : 6 * N);
    static constexpr int CPW = 64 / LPC;                       // cells per wave
    static constexpr int GS = (36 * NF > 3 * ND) ? 36 * NF : 3 * ND;  // work area per cell
    static_assert(NF <= 64 && 6 * N <= 64, "one wave per cell at most");
};

// local index with coordinate m along direction d and (p, r) along the two
// other directions in increasing order
template <int N>
__device__ __forceinline__ int lix(int d, int m, int p, int r)
{
    return d == 0 ? m + N * (p + N * r) : (d == 1 ? p + N * (m + N * r) : p + N * (r + N * m));
}

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    return __builtin_nontemporal_load(p);
}

template <int N, typename T>
__global__ void __launch_bounds__(64)
k_apply(const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ bvec,
        const T *__restrict__ cell, const T *__restrict__ face, const int32_t *__restrict__ nbr,
        const int32_t *__restrict__ order, int n_cells, int nwg)
{
    constexpr int NF = Cfg<N>::NF, ND = Cfg<N>::ND, LPC = Cfg<N>::LPC, CPW = Cfg<N>::CPW,
                  GS = Cfg<N>::GS;
    __shared__ T sU[CPW][ND];
    __shared__ T sG[CPW][GS];

    // contiguous ranges of the traversal per XCD (workgroups are dealt
    // round-robin to the XCDs)
    const int bid = blockIdx.x;
    const int q8 = nwg / NXCD, r8 = nwg % NXCD, xcd = bid % NXCD;
    const int wg = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / NXCD;

    const int lane = threadIdx.x;
    const int cs = lane / LPC;             // cell slot in the wave
    const int ln = lane - cs * LPC;        // lane within the cell
    const int slot = wg * CPW + cs;
    const bool valid = slot < n_cells;
    const int64_t cid = valid ? order[slot] : 0;
    T *G = &sG[cs][0];
    T *U = &sU[cs][0];

    // ---- cell lanes: (a, b), pencil owners
    const bool cl = valid && ln < NF;
    const int a = ln % N, b = (ln / N) % N;
    // ---- face lanes: (f, p), column owners
    const bool fl0 = valid && ln < 6 * N;
    const int f = fl0 ? ln / N : 0, rr = ln % N;
    const int d = f >> 1, s = f & 1;
    const int32_t nb = fl0 ? nbr[cid * 6 + f] : -1;
    const bool fl = nb >= 0;

    if (valid)
        for (int e = ln; e < ND; e += LPC) sU[cs][e] = x[cid * ND + e];

    // the neighbour's layer values and normal derivatives on column p of face
    // f, loaded with the own values so that both arrive in one memory round
    // trip; the N lanes of a face read neighbouring addresses in each load
    T Ln[N], Nn[N];
    if (fl) {
        const int en = 1 - s, mn = en ? N - 1 : 0;
        const T *xn = x + (int64_t)nb * ND;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            T sn = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) sn += tE<T, N>(en, m) * xn[lix<N>(d, m, rr, r)];
            Nn[r] = sn;
            Ln[r] = xn[lix<N>(d, mn, rr, r)];
        }
    }

    // quadrature-point data of this lane's z pencil, streamed once
    const T *cp = cell + cid * 7 * ND + a + N * b;
    __syncthreads();

    T Y[N];
    // =========================================================== cell part
    // x sweep: lane (j=a, l=b): B u and BD u along x
    if (cl) {
        T r[N];
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = U[i + N * a + NF * b];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            T s0 = 0, s1 = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                s0 += tB<T, N>(q, i) * r[i];
                s1 += tD<T, N>(q, i) * r[i];
            }
            G[q + N * a + NF * b] = s0;
            G[ND + q + N * a + NF * b] = s1;
        }
    }
    __syncthreads();
    // y sweep: lane (qx=a, l=b)
    {
        T c0[N], c1[N], c2[N];
        if (cl) {
            T p0[N], p1[N];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                p0[j] = G[a + N * j + NF * b];
                p1[j] = G[ND + a + N * j + NF * b];
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
        if (cl) {
#pragma unroll
            for (int q = 0; q < N; ++q) {
                G[a + N * q + NF * b] = c0[q];            // u
                G[ND + a + N * q + NF * b] = c1[q];       // d/deta
                G[2 * ND + a + N * q + NF * b] = c2[q];   // d/dxi
            }
        }
    }
    __syncthreads();
    // z sweep, quadrature-point operation and transposed z sweep: lane (qx=a, qy=b)
    {
        T t0[N], t1[N], t2[N];
        if (cl) {
            T p0[N], p1[N], p2[N];
#pragma unroll
            for (int l = 0; l < N; ++l) {
                p0[l] = G[a + N * b + NF * l];
                p1[l] = G[ND + a + N * b + NF * l];
                p2[l] = G[2 * ND + a + N * b + NF * l];
                t0[l] = t1[l] = t2[l] = 0;
            }
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
                const T *cq = cp + NF * q;
                const T m = ld_stream(cq), gxx = ld_stream(cq + ND), gxy = ld_stream(cq + 2 * ND),
                        gxz = ld_stream(cq + 3 * ND), gyy = ld_stream(cq + 4 * ND),
                        gyz = ld_stream(cq + 5 * ND), gzz = ld_stream(cq + 6 * ND);
                const T v = m * u;
                const T fx = gxx * dx + gxy * dy + gxz * dz;
                const T fy = gxy * dx + gyy * dy + gyz * dz;
                const T fz = gxz * dx + gyz * dy + gzz * dz;
#pragma unroll
                for (int l = 0; l < N; ++l) {
                    t0[l] += tB<T, N>(q, l) * v + tD<T, N>(q, l) * fz;
                    t1[l] += tB<T, N>(q, l) * fy;
                    t2[l] += tB<T, N>(q, l) * fx;
                }
            }
        }
        __syncthreads();
        if (cl) {
#pragma unroll
            for (int l = 0; l < N; ++l) {
                G[a + N * b + NF * l] = t0[l];
                G[ND + a + N * b + NF * l] = t1[l];
                G[2 * ND + a + N * b + NF * l] = t2[l];
            }
        }
    }
    __syncthreads();
    // transposed y sweep: lane (qx=a, l=b)
    {
        T s0v[N], s1v[N];
        if (cl) {
            T p0[N], p1[N], p2[N];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                p0[q] = G[a + N * q + NF * b];
                p1[q] = G[ND + a + N * q + NF * b];
                p2[q] = G[2 * ND + a + N * q + NF * b];
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
        if (cl) {
#pragma unroll
            for (int j = 0; j < N; ++j) {
                G[a + N * j + NF * b] = s0v[j];
                G[ND + a + N * j + NF * b] = s1v[j];
            }
        }
    }
    __syncthreads();
    // transposed x sweep: lane (j=a, l=b) keeps its output pencil in Y
    if (cl) {
        T p0[N], p1[N];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            p0[q] = G[q + N * a + NF * b];
            p1[q] = G[ND + q + N * a + NF * b];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T sacc = 0;
#pragma unroll
            for (int q = 0; q < N; ++q) sacc += tB<T, N>(q, i) * p0[q] + tD<T, N>(q, i) * p1[q];
            Y[i] = sacc;
        }
    }
    __syncthreads();

    // =========================================================== face part
    // step 1, lane (f, p): own layer and normal derivative on column p (the
    // neighbour's were formed at the start), then interpolation of both sides
    // along the second tangential direction
    if (fl) {
        const int eo = s, mo = eo ? N - 1 : 0;
        T Lo[N], No[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            T so = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) so += tE<T, N>(eo, m) * U[lix<N>(d, m, rr, r)];
            No[r] = so;
            Lo[r] = U[lix<N>(d, mo, rr, r)];
        }
        T *gw = G + f * 6 * NF + rr;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            T g0 = 0, g1 = 0, g2 = 0, g3 = 0, g4 = 0, g5 = 0;
#pragma unroll
            for (int r = 0; r < N; ++r) {
                const T bb = tB<T, N>(q, r), bd = tD<T, N>(q, r);
                g0 += bb * Lo[r]; g1 += bd * Lo[r]; g2 += bb * No[r];
                g3 += bb * Ln[r]; g4 += bd * Ln[r]; g5 += bb * Nn[r];
            }
            gw[0 * NF + q * N] = g0; gw[1 * NF + q * N] = g1; gw[2 * NF + q * N] = g2;
            gw[3 * NF + q * N] = g3; gw[4 * NF + q * N] = g4; gw[5 * NF + q * N] = g5;
        }
    }
    __syncthreads();
    // the own values are no longer needed: the output pencils wait in sU
    if (cl) {
#pragma unroll
        for (int i = 0; i < N; ++i) sU[cs][i + N * a + NF * b] = Y[i];
    }
    // step 2, lane (f, q2): first tangential direction, flux terms at the
    // Gauss points, transposed sweep back along it.  The neighbour side is
    // evaluated first (its flux and value per point), then the own side.
    {
        T A0[N], A1[N], A2[N];
        const int q2 = rr;
        if (fl) {
            const int64_t fid = s ? cid : (int64_t)nb;
            const T *fd = face + (fid * 3 + d) * 7 * NF + q2;   // [comp][q1][q2]
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            const T *gr = G + f * 6 * NF + q2 * N;
            // g of the neighbour side: g+ if the own cell is the minus cell
            const int gn_off = s ? 3 : 0, go_off = s ? 0 : 3;
            T fnb[N], vnb[N];
            {
                T h0[N], h1[N], h2[N];
#pragma unroll
                for (int p = 0; p < N; ++p) {
                    h0[p] = gr[3 * NF + p];
                    h1[p] = gr[4 * NF + p];
                    h2[p] = gr[5 * NF + p];
                }
#pragma unroll
                for (int q1 = 0; q1 < N; ++q1) {
                    T vn = 0, t1n = 0, t2n = 0, dnn = 0;
#pragma unroll
                    for (int p = 0; p < N; ++p) {
                        const T bb = tB<T, N>(q1, p), bd = tD<T, N>(q1, p);
                        vn += bb * h0[p]; t1n += bd * h0[p]; t2n += bb * h1[p]; dnn += bb * h2[p];
                    }
                    const T *fq = fd + N * q1 + gn_off * NF;
                    T gn[3];
                    gn[d] = dnn; gn[t1] = t1n; gn[t2] = t2n;
                    fnb[q1] = fq[0] * gn[0] + fq[NF] * gn[1] + fq[2 * NF] * gn[2];
                    vnb[q1] = vn;
                }
            }
            T h0[N], h1[N], h2[N];
#pragma unroll
            for (int p = 0; p < N; ++p) {
                h0[p] = gr[p];
                h1[p] = gr[NF + p];
                h2[p] = gr[2 * NF + p];
                A0[p] = A1[p] = A2[p] = 0;
            }
#pragma unroll
            for (int q1 = 0; q1 < N; ++q1) {
                T vo = 0, t1o = 0, t2o = 0, dno = 0;
#pragma unroll
                for (int p = 0; p < N; ++p) {
                    const T bb = tB<T, N>(q1, p), bd = tD<T, N>(q1, p);
                    vo += bb * h0[p]; t1o += bd * h0[p]; t2o += bb * h1[p]; dno += bb * h2[p];
                }
                const T *fq = fd + N * q1 + go_off * NF;
                const T g0 = fq[0], g1 = fq[NF], g2 = fq[2 * NF];
                const T pen = fd[6 * NF + N * q1];
                T go[3];
                go[d] = dno; go[t1] = t1o; go[t2] = t2o;
                const T flux = g0 * go[0] + g1 * go[1] + g2 * go[2] + fnb[q1];
                const T jump = s ? (vo - vnb[q1]) : (vnb[q1] - vo);
                const T sg = s ? T(1) : T(-1);
                const T cv = sg * (T(-0.5) * flux + pen * jump);
                const T hj = T(-0.5) * jump;
                T cg[3] = {hj * g0, hj * g1, hj * g2};
                const T ct1 = cg[t1], ct2 = cg[t2], cn = cg[d];
#pragma unroll
                for (int p = 0; p < N; ++p) {
                    const T bb = tB<T, N>(q1, p), bd = tD<T, N>(q1, p);
                    A0[p] += bb * cv + bd * ct1;
                    A1[p] += bb * ct2;
                    A2[p] += bb * cn;
                }
            }
        }
        __syncthreads();
        if (fl) {
            T *gw = G + f * 3 * NF + q2 * N;
#pragma unroll
            for (int p = 0; p < N; ++p) {
                gw[p] = A0[p];
                gw[NF + p] = A1[p];
                gw[2 * NF + p] = A2[p];
            }
        }
    }
    __syncthreads();
    // step 3, lane (f, p): transposed sweep along the second tangential
    // direction; the layer (F0) and normal-derivative (F1) weights of column p
    if (fl0) {
        T *out = G + 18 * NF + f * 2 * NF + rr;      // [field][r][p]
        if (fl) {
            const T *gr = G + f * 3 * NF + rr;
            T h0[N], h1[N], h2[N];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                h0[q] = gr[q * N];
                h1[q] = gr[NF + q * N];
                h2[q] = gr[2 * NF + q * N];
            }
#pragma unroll
            for (int r = 0; r < N; ++r) {
                T f0 = 0, f1 = 0;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    f0 += tB<T, N>(q, r) * h0[q] + tD<T, N>(q, r) * h1[q];
                    f1 += tB<T, N>(q, r) * h2[q];
                }
                out[r * N] = f0;
                out[NF + r * N] = f1;
            }
        } else {
#pragma unroll
            for (int r = 0; r < N; ++r) out[r * N] = out[NF + r * N] = 0;
        }
    }
    __syncthreads();
    // pencil owners (j=a, l=b) add the six faces' contributions
    if (cl) {
#pragma unroll
        for (int i = 0; i < N; ++i) Y[i] = sU[cs][i + N * a + NF * b];
        const T *F = G + 18 * NF;
        // x faces: normal coordinate i, (p, r) = (j, l)
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
            const T f0 = F[(0 + sx) * 2 * NF + b * N + a], f1 = F[(0 + sx) * 2 * NF + NF + b * N + a];
#pragma unroll
            for (int i = 0; i < N; ++i)
                Y[i] += tE<T, N>(sx, i) * f1 + ((i == (sx ? N - 1 : 0)) ? f0 : T(0));
        }
        // y faces: normal coordinate j = a, (p, r) = (i, l)
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            const T *F0 = F + (2 + sy) * 2 * NF + b * N, *F1 = F0 + NF;
            T e1 = 0;
            // DL[sy][a] with a lane-dependent index: unrolled select
#pragma unroll
            for (int m = 0; m < N; ++m)
                if (m == a) e1 = tE<T, N>(sy, m);
            const bool on = a == (sy ? N - 1 : 0);
#pragma unroll
            for (int i = 0; i < N; ++i) Y[i] += e1 * F1[i] + (on ? F0[i] : T(0));
        }
        // z faces: normal coordinate l = b, (p, r) = (i, j)
#pragma unroll
        for (int sz = 0; sz < 2; ++sz) {
            const T *F0 = F + (4 + sz) * 2 * NF + a * N, *F1 = F0 + NF;
            T e1 = 0;
#pragma unroll
            for (int m = 0; m < N; ++m)
                if (m == b) e1 = tE<T, N>(sz, m);
            const bool on = b == (sz ? N - 1 : 0);
#pragma unroll
            for (int i = 0; i < N; ++i) Y[i] += e1 * F1[i] + (on ? F0[i] : T(0));
        }
        const int64_t o = cid * ND + N * a + NF * b;
#pragma unroll
        for (int i = 0; i < N; ++i) y[o + i] = bvec ? bvec[o + i] - Y[i] : Y[i];
    }
}

template <int N, typename T>
hipError_t apply_n(hx_ctx *c, const T *x, T *y, const T *b)
{
    const int cpw = Cfg<N>::CPW;
    const int nwg = (int)((c->n_cells + cpw - 1) / cpw);
    const T *cell = std::is_same<T, double>::value ? (const T *)c->cell64 : (const T *)c->cell32;
    const T *face = std::is_same<T, double>::value ? (const T *)c->face64 : (const T *)c->face32;
    hipLaunchKernelGGL((k_apply<N, T>), dim3(nwg), dim3(64), 0, c->stream, x, y, b, cell, face,
                       c->nbr, c->order, (int)c->n_cells, nwg);
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
