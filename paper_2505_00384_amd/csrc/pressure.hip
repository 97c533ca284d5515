// The pressure system of one IMEX stage (paper section 2: the discrete
// momentum and energy equations A U + B P = F, C U + D P = G, and the system
// D P + C A^-1 (F - B P) = G solved for the pressure).  The paper names the
// matrices without giving them; with central fluxes they are
//   (B p)_{e,i} = tau [ -int_K p d_e phi_i + int_dK p^ phi_i n_{K,e} ],
//       p^ = {p} on interior faces, the own trace on boundary faces;
//   (C u)_i     = tau [ -int_K hr u . grad Psi_i + int_dK {hr u . n_K} Psi_i ],
//       interior faces only (no flux through the boundary);
//   A = rho-weighted velocity mass (one scalar block per component),
//   D = (1/(gamma - 1)) mass (internal energy of an ideal gas),
// with hr = h rho and (k+1)-point Gauss rules on cells and faces, the rule of
// the fast block-diagonal inverse (section 3.3), so A^-1 is exact by the
// tensor-product sweeps of k_massinv.
//
// k_grad and k_div: NF threads per cell (pencil owners (a, b)), CPB cells
// per block (k_grad: one wave, so its LDS exchanges need no workgroup
// barrier; k_div: two waves, measured faster with its larger LDS), cells taken in the operator's tile traversal with one contiguous range of
// blocks per XCD, so neighbours' data are found in the same L2.  Cell terms by sum factorisation: values at the Gauss points by
// three sweeps, the pointwise metric terms W = w detJ J^-1 (times hr for C),
// and the transposed gradient (B^T / BD^T sweeps z, y, x).  Face terms: the
// traces at the face Gauss points are N x N contractions of the face layers
// (GLL nodes include the faces), the transposed contraction returns them to
// the face-layer nodes, and the pencil owners add them.  Each output is
// written by one thread: no atomics, bitwise reproducible.
#include "common.hpp"

namespace hx {
namespace {

// compile-time 1-D tables (generated at build time from the library's rules,
// the same values as the reference tables): in unrolled loops their entries
// become instruction operands instead of memory reads
template <int N> struct KB;
template <int N> struct KBD;
template <int N> struct KDL;
#include "optables.inc"
template <int N> struct KBI;
#include "optables_binv.inc"

template <int N>
__device__ __forceinline__ constexpr double tB(int q, int i) { return KB<N>::d[q * N + i]; }
template <int N>
__device__ __forceinline__ constexpr double tD(int q, int i) { return KBD<N>::d[q * N + i]; }
// (B^-1)_{iq}: B maps nodes to Gauss points and is square
template <int N>
__device__ __forceinline__ constexpr double tBi(int i, int q) { return KBI<N>::d[i * N + q]; }

// CPB cells of NF threads per block of at most TMAX threads (k_grad: one
// wave; k_div, with three velocity components in LDS: two waves)
template <int N, int TMAX>
struct PCfg {
    static constexpr int NF = N * N, ND = N * N * N;
    static constexpr int CPB = (TMAX / NF) > 0 ? TMAX / NF : 1;
    static constexpr int NT = ((CPB * NF + 63) / 64) * 64;
};
constexpr int GRAD_T = 64, DIV_T = 128;
template <int N> constexpr int grad_nt() { return PCfg<N, GRAD_T>::NT; }
template <int N> constexpr int div_nt() { return PCfg<N, DIV_T>::NT; }

// cell-local index of face-layer node (e1, e2) at normal coordinate m of
// direction d; e1, e2 run along the tangential directions t1 < t2
template <int N>
__device__ __forceinline__ int lay(int d, int m, int e1, int e2)
{
    const int s1 = d == 0 ? N : 1, s2 = d == 2 ? N : N * N, sd = d == 0 ? 1 : (d == 1 ? N : N * N);
    return m * sd + e1 * s1 + e2 * s2;
}

// per-lane rows and columns of B for the face contractions of lane (a, b):
// Ra[e] = B(a, e), Rb[e] = B(b, e), Ca[e] = B(e, a), Cb[e] = B(e, b)
template <int N>
struct LaneB {
    double Ra[N], Rb[N], Ca[N], Cb[N];
    __device__ __forceinline__ LaneB(const double *sB, int a, int b)
    {
#pragma unroll
        for (int e = 0; e < N; ++e) {
            Ra[e] = sB[a * N + e];
            Rb[e] = sB[b * N + e];
            Ca[e] = sB[e * N + a];
            Cb[e] = sB[e * N + b];
        }
    }
};

// value of a face layer at the lane's face Gauss point (a, b):
// sum B(a,e1) B(b,e2) v(e1, e2), the layer at normal coordinate m of d
template <int N>
__device__ __forceinline__ double trace_at(const LaneB<N> &L, const double *v, int d, int m)
{
    double s = 0.0;
#pragma unroll
    for (int e2 = 0; e2 < N; ++e2) {
        double r = 0.0;
#pragma unroll
        for (int e1 = 0; e1 < N; ++e1) r += L.Ra[e1] * v[lay<N>(d, m, e1, e2)];
        s += L.Rb[e2] * r;
    }
    return s;
}

// the same from a face layer already gathered as v[e1 + N e2]
template <int N>
__device__ __forceinline__ double trace_at2(const LaneB<N> &L, const double *v)
{
    double s = 0.0;
#pragma unroll
    for (int e2 = 0; e2 < N; ++e2) {
        double r = 0.0;
#pragma unroll
        for (int e1 = 0; e1 < N; ++e1) r += L.Ra[e1] * v[e1 + N * e2];
        s += L.Rb[e2] * r;
    }
    return s;
}

// transposed contraction of a face field g[a' + N b'] to the lane's node
// (e1, e2) = (a, b)
template <int N>
__device__ __forceinline__ double trace_t(const LaneB<N> &L, const double *g)
{
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
        double r = 0.0;
#pragma unroll
        for (int a = 0; a < N; ++a) r += L.Ca[a] * g[a + N * b];
        s += L.Cb[b] * r;
    }
    return s;
}

// values of a cell field at the Gauss points along the lane's z pencil
// (lane (a, b) = (qx, qy)); v is the field in LDS, F a scratch field
template <int N>
__device__ __forceinline__ void to_gauss(const double *v, double *F, bool act, int a, int b,
                                         double (&out)[N])
{
    constexpr int NF = N * N;
    double r[N], w[N];
    if (act) {
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = v[i + N * a + NF * b];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < N; ++i) s += tB<N>(q, i) * r[i];
            w[q] = s;
        }
#pragma unroll
        for (int q = 0; q < N; ++q) F[q + N * a + NF * b] = w[q];
    }
    __syncthreads();
    if (act) {
#pragma unroll
        for (int j = 0; j < N; ++j) r[j] = F[a + N * j + NF * b];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += tB<N>(q, j) * r[j];
            w[q] = s;
        }
    }
    __syncthreads();
    if (act)
#pragma unroll
        for (int q = 0; q < N; ++q) F[a + N * q + NF * b] = w[q];
    __syncthreads();
    if (act) {
#pragma unroll
        for (int l = 0; l < N; ++l) r[l] = F[a + N * b + NF * l];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < N; ++l) s += tB<N>(q, l) * r[l];
            out[q] = s;
        }
    }
    __syncthreads();
}

// y = -tau sum_d G_d^T t_d, G_d the reference gradient component d at the
// Gauss points; t_d given along the lane's z pencil; F0..F2 scratch fields;
// the result is the lane's x pencil (lane (a, b) = (j, l))
template <int N>
__device__ __forceinline__ void grad_t(double *F0, double *F1, double *F2, bool act, int a, int b,
                                       const double (&t0)[N], const double (&t1)[N],
                                       const double (&t2)[N], double tau, double (&y)[N])
{
    constexpr int NF = N * N;
    if (act) {
#pragma unroll
        for (int l = 0; l < N; ++l) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                s0 += tB<N>(q, l) * t0[q];
                s1 += tB<N>(q, l) * t1[q];
                s2 += tD<N>(q, l) * t2[q];
            }
            F0[a + N * b + NF * l] = s0;
            F1[a + N * b + NF * l] = s1;
            F2[a + N * b + NF * l] = s2;
        }
    }
    __syncthreads();
    double r0[N], r12[N];
    if (act) {
        double f0[N], f1[N], f2[N];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            f0[q] = F0[a + N * q + NF * b];
            f1[q] = F1[a + N * q + NF * b];
            f2[q] = F2[a + N * q + NF * b];
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double s0 = 0.0, s12 = 0.0;
#pragma unroll
            for (int q = 0; q < N; ++q) {
                s0 += tB<N>(q, j) * f0[q];
                s12 += tD<N>(q, j) * f1[q] + tB<N>(q, j) * f2[q];
            }
            r0[j] = s0;
            r12[j] = s12;
        }
    }
    __syncthreads();
    if (act)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            F0[a + N * j + NF * b] = r0[j];
            F1[a + N * j + NF * b] = r12[j];
        }
    __syncthreads();
    if (act) {
        double g0[N], g1[N];
#pragma unroll
        for (int q = 0; q < N; ++q) {
            g0[q] = F0[q + N * a + NF * b];
            g1[q] = F1[q + N * a + NF * b];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < N; ++q) s += tD<N>(q, i) * g0[q] + tB<N>(q, i) * g1[q];
            y[i] = -tau * s;
        }
    }
    __syncthreads();
}

// M^{-1} y for three fields at once, M = B3^T diag(m) B3 the cell mass block
// with Gauss-point weights m (m[a + N b + N^2 q] for the lane's z pencil):
// y holds the lane's x pencils (lane (a, b) = (j, l)) on entry and on exit;
// F[0..2] are scratch fields
template <int N>
__device__ __forceinline__ void mass_inv3(double *F0, double *F1, double *F2, bool act, int a, int b,
                                          const double *m, double (&y)[3][N])
{
    constexpr int NF = N * N;
    double *F[3] = {F0, F1, F2};
    // B^-T along x, in registers
    if (act)
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int q = 0; q < N; ++q) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < N; ++i) s += tBi<N>(i, q) * y[e][i];
                F[e][q + N * a + NF * b] = s;
            }
    __syncthreads();
    // B^-T along y: lane (qx=a, l=b)
    double w[3][N];
    if (act)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            double v[N];
#pragma unroll
            for (int j = 0; j < N; ++j) v[j] = F[e][a + N * j + NF * b];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < N; ++j) s += tBi<N>(j, q) * v[j];
                w[e][q] = s;
            }
        }
    __syncthreads();
    if (act)
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int q = 0; q < N; ++q) F[e][a + N * q + NF * b] = w[e][q];
    __syncthreads();
    // B^-T along z, 1/m, B^-1 along z: lane (qx=a, qy=b)
    if (act) {
        double mi[N];
#pragma unroll
        for (int q = 0; q < N; ++q) mi[q] = 1.0 / m[NF * q];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            double v[N], t[N];
#pragma unroll
            for (int l = 0; l < N; ++l) v[l] = F[e][a + N * b + NF * l];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                double s = 0.0;
#pragma unroll
                for (int l = 0; l < N; ++l) s += tBi<N>(l, q) * v[l];
                t[q] = s * mi[q];
            }
#pragma unroll
            for (int l = 0; l < N; ++l) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < N; ++q) s += tBi<N>(l, q) * t[q];
                w[e][l] = s;
            }
        }
    }
    __syncthreads();
    if (act)
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int l = 0; l < N; ++l) F[e][a + N * b + NF * l] = w[e][l];
    __syncthreads();
    // B^-1 along y: lane (qx=a, l=b)
    if (act)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            double v[N];
#pragma unroll
            for (int q = 0; q < N; ++q) v[q] = F[e][a + N * q + NF * b];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < N; ++q) s += tBi<N>(j, q) * v[q];
                w[e][j] = s;
            }
        }
    __syncthreads();
    if (act)
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
            for (int j = 0; j < N; ++j) F[e][a + N * j + NF * b] = w[e][j];
    __syncthreads();
    // B^-1 along x: lane (j=a, l=b), back into y
    if (act)
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            double v[N];
#pragma unroll
            for (int q = 0; q < N; ++q) v[q] = F[e][q + N * a + NF * b];
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double s = 0.0;
#pragma unroll
                for (int q = 0; q < N; ++q) s += tBi<N>(i, q) * v[q];
                y[e][i] = s;
            }
        }
    __syncthreads();
}

// y = B3^T t: transposed interpolation of Gauss-point values t (the lane's
// z pencil) back to the nodes (the lane's x pencil); F a scratch field
template <int N>
__device__ __forceinline__ void interp_t(double *F, bool act, int a, int b, const double (&t)[N],
                                         double (&y)[N])
{
    constexpr int NF = N * N;
    if (act)
#pragma unroll
        for (int l = 0; l < N; ++l) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < N; ++q) s += tB<N>(q, l) * t[q];
            F[a + N * b + NF * l] = s;
        }
    __syncthreads();
    double r[N];
    if (act)
#pragma unroll
        for (int j = 0; j < N; ++j) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < N; ++q) s += tB<N>(q, j) * F[a + N * q + NF * b];
            r[j] = s;
        }
    __syncthreads();
    if (act)
#pragma unroll
        for (int j = 0; j < N; ++j) F[a + N * j + NF * b] = r[j];
    __syncthreads();
    if (act)
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < N; ++q) s += tB<N>(q, i) * F[q + N * a + NF * b];
            y[i] = s;
        }
    __syncthreads();
}

// add face-layer contributions A[f][e1 + N e2] of the six faces to the x
// pencil (i, j=a, l=b) of the lane
// add the contribution of face f, computed on its face layer (e1, e2), to
// the pencil y of lane (a, b): x faces hold nodes (0 or N-1, a, b) with
// (e1, e2) = (j, l); y faces j = a with (e1, e2) = (i, l); z faces l = b with
// (e1, e2) = (i, j)
template <int N>
__device__ __forceinline__ void add_face(const double *A, int f, int a, int b, double (&y)[N])
{
    switch (f) {
    case 0: y[0] += A[a + N * b]; break;
    case 1: y[N - 1] += A[a + N * b]; break;
    case 2: if (a == 0) for (int i = 0; i < N; ++i) y[i] += A[i + N * b]; break;
    case 3: if (a == N - 1) for (int i = 0; i < N; ++i) y[i] += A[i + N * b]; break;
    case 4: if (b == 0) for (int i = 0; i < N; ++i) y[i] += A[i + N * a]; break;
    default: if (b == N - 1) for (int i = 0; i < N; ++i) y[i] += A[i + N * a]; break;
    }
}

// MINV: the output is A^-1 B p (the rho-weighted mass inverse of each
// component applied in the epilogue, weights mr), else B p
template <int N, bool MINV>
__global__ void __launch_bounds__(grad_nt<N>())
k_grad(const double *__restrict__ p, double *__restrict__ u3, int64_t nt,
       const double *__restrict__ W, const double *__restrict__ fn, const int32_t *__restrict__ visit,
       const RefTab64 *__restrict__ T, double tau, int n_cells, int nwg,
       const double *__restrict__ mr)
{
    constexpr int NF = PCfg<N, GRAD_T>::NF, ND = PCfg<N, GRAD_T>::ND, CPB = PCfg<N, GRAD_T>::CPB;
    __shared__ double sB[NF];
    __shared__ double sP[CPB][ND];
    __shared__ double sF[CPB][3][ND];
    __shared__ double sG[CPB][3][NF];
    __shared__ double sA[CPB][3][NF];
    __shared__ double sL[CPB][NF];
    const int t = threadIdx.x;
    const int lc0 = t / NF;
    const bool slot = lc0 < CPB;
    const int lc = slot ? lc0 : 0;
    const int tt = t - lc0 * NF;
    const int a = tt % N, b = tt / N;
    // the operator's traversal: slot records {cell, six neighbours} in tile
    // order, one contiguous range of blocks per XCD
    const int bid = blockIdx.x;
    const int q8 = nwg / NXCD, r8 = nwg % NXCD, xcd = bid % NXCD;
    const int wg = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / NXCD;
    const int64_t sl = (int64_t)wg * CPB + lc;
    const bool act = slot && sl < n_cells;
    // the 32-byte record in two 16-byte loads (slot 0's for idle threads)
    const int4 *rec4 = reinterpret_cast<const int4 *>(visit + (act ? sl : 0) * 8);
    const int4 r0 = rec4[0], r1 = rec4[1];
    const int32_t nbr6[6] = {r0.y, r0.z, r0.w, r1.x, r1.y, r1.z};
    const int64_t cid = act ? r0.x : 0;

    // one batch of loads (one memory round trip): the 1-D table, the cell's
    // values, the neighbours' face layers (one value per lane and face; a
    // missing neighbour reads the own cell and is dropped) and the first
    // face's outward ds n; they are requested before the cell part so that
    // their latency overlaps it
    static_assert(NF <= PCfg<N, GRAD_T>::NT, "one table entry per thread");
    const double fbv = t < NF ? T->B[t] : 0.0;
    double pv[N], nbv[6], fnx[3];
#pragma unroll
    for (int u = 0; u < N; ++u) pv[u] = p[cid * ND + tt + u * NF];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int32_t nb = act ? nbr6[f] : -1;
        const int64_t src = nb >= 0 ? (int64_t)nb : cid;
        const double v = p[src * ND + lay<N>(f >> 1, (f & 1) ? 0 : N - 1, a, b)];
        nbv[f] = nb >= 0 ? v : 0.0;
    }
#pragma unroll
    for (int ec = 0; ec < 3; ++ec) fnx[ec] = fn[(cid * 6 + 0) * 3 * NF + tt + ec * NF];
    __builtin_amdgcn_sched_barrier(0);
    if (t < NF) sB[t] = fbv;
    if (act) {
#pragma unroll
        for (int u = 0; u < N; ++u) sP[lc][tt + u * NF] = pv[u];
    }
    __syncthreads();
    const LaneB<N> LB(sB, a, b);
    double pq[N];
    to_gauss<N>(sP[lc], sF[lc][0], act, a, b, pq);
    double Y[3][N];
#pragma unroll
    for (int ec = 0; ec < 3; ++ec) {
        double t0[N], t1[N], t2[N];
        if (act) {
            const double *Wc = W + cid * 9 * ND + a + N * b;
            for (int q = 0; q < N; ++q) {
                t0[q] = pq[q] * Wc[(0 + ec) * ND + NF * q];
                t1[q] = pq[q] * Wc[(3 + ec) * ND + NF * q];
                t2[q] = pq[q] * Wc[(6 + ec) * ND + NF * q];
            }
        }
        grad_t<N>(sF[lc][0], sF[lc][1], sF[lc][2], act, a, b, t0, t1, t2, tau, Y[ec]);
    }
    // faces: tau ds n_e p^ at the Gauss points, back to the face-layer nodes;
    // the neighbour's face layer is gathered into LDS first (one value per lane)
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, s = f & 1;
        const int32_t nb = act ? nbr6[f] : -1;
        // this face's ds n, and the next face's requested now
        double fcur[3];
#pragma unroll
        for (int ec = 0; ec < 3; ++ec) fcur[ec] = fnx[ec];
        if (f < 5) {
#pragma unroll
            for (int ec = 0; ec < 3; ++ec) fnx[ec] = fn[(cid * 6 + f + 1) * 3 * NF + tt + ec * NF];
        }
        if (nb >= 0) sL[lc][tt] = nbv[f];
        __syncthreads();
        if (act) {
            const double po = trace_at<N>(LB, sP[lc], d, s ? N - 1 : 0);
            double ph = po;
            if (nb >= 0) ph = 0.5 * (po + trace_at2<N>(LB, sL[lc]));
            for (int ec = 0; ec < 3; ++ec) sG[lc][ec][tt] = tau * ph * fcur[ec];
        }
        __syncthreads();
        if (act)
            for (int ec = 0; ec < 3; ++ec) sA[lc][ec][tt] = trace_t<N>(LB, sG[lc][ec]);
        __syncthreads();
        if (act)
#pragma unroll
            for (int ec = 0; ec < 3; ++ec) add_face<N>(sA[lc][ec], f, a, b, Y[ec]);
    }
    if (MINV)
        mass_inv3<N>(sF[lc][0], sF[lc][1], sF[lc][2], act, a, b, mr + cid * ND + a + N * b, Y);
    if (act)
#pragma unroll
        for (int ec = 0; ec < 3; ++ec) {
            const int64_t o = ec * nt + cid * ND + N * a + NF * b;
            for (int i = 0; i < N; ++i) u3[o + i] = Y[ec][i];
        }
}

// DP: the output is D x - C u (or bv - (D x - C u) when bv is given), with
// D the mass of Gauss-point weights md, else C u
template <int N, bool DP>
__global__ void __launch_bounds__(div_nt<N>())
k_div(const double *__restrict__ u3, double *__restrict__ qv, int64_t nt,
      const double *__restrict__ WC, const double *__restrict__ fn, const double *__restrict__ fh,
      const int32_t *__restrict__ visit, const RefTab64 *__restrict__ T, double tau, int n_cells, int nwg,
      const double *__restrict__ xv, const double *__restrict__ md, const double *__restrict__ bv)
{
    constexpr int NF = PCfg<N, DIV_T>::NF, ND = PCfg<N, DIV_T>::ND, CPB = PCfg<N, DIV_T>::CPB;
    __shared__ double sB[NF];
    __shared__ double sU[CPB][3][ND];
    __shared__ double sF[CPB][ND];
    __shared__ double sG[CPB][NF];
    __shared__ double sA[CPB][NF];
    __shared__ double sL[CPB][3][NF];
    const int t = threadIdx.x;
    const int lc0 = t / NF;
    const bool slot = lc0 < CPB;
    const int lc = slot ? lc0 : 0;
    const int tt = t - lc0 * NF;
    const int a = tt % N, b = tt / N;
    // the operator's traversal: slot records {cell, six neighbours} in tile
    // order, one contiguous range of blocks per XCD
    const int bid = blockIdx.x;
    const int q8 = nwg / NXCD, r8 = nwg % NXCD, xcd = bid % NXCD;
    const int wg = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / NXCD;
    const int64_t sl = (int64_t)wg * CPB + lc;
    const bool act = slot && sl < n_cells;
    // the 32-byte record in two 16-byte loads (slot 0's for idle threads)
    const int4 *rec4 = reinterpret_cast<const int4 *>(visit + (act ? sl : 0) * 8);
    const int4 r0 = rec4[0], r1 = rec4[1];
    const int32_t nbr6[6] = {r0.y, r0.z, r0.w, r1.x, r1.y, r1.z};
    const int64_t cid = act ? r0.x : 0;

    // one batch of loads (one memory round trip): the 1-D table, the cell's
    // three velocity components, the neighbours' face layers of the three
    // (a missing neighbour reads the own cell and is dropped) and the first
    // face's ds n and h rho factors
    static_assert(NF <= PCfg<N, DIV_T>::NT, "one table entry per thread");
    const double fbv = t < NF ? T->B[t] : 0.0;
    double uv[3][N], nbu[6][3], fnx[3], fhx[2];
#pragma unroll
    for (int ec = 0; ec < 3; ++ec)
#pragma unroll
        for (int u = 0; u < N; ++u) uv[ec][u] = u3[ec * nt + cid * ND + tt + u * NF];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int32_t nb = act ? nbr6[f] : -1;
        const int64_t src = nb >= 0 ? (int64_t)nb : cid;
        const int64_t o = src * ND + lay<N>(f >> 1, (f & 1) ? 0 : N - 1, a, b);
#pragma unroll
        for (int ec = 0; ec < 3; ++ec) nbu[f][ec] = u3[ec * nt + o];
    }
    // ds n and the two h rho factors of face f (the neighbour's entry of a
    // missing neighbour reads the own cell's and is not used)
    auto face_data = [&](int f, double (&fo)[3], double (&ho)[2]) {
        const int32_t nb = act ? nbr6[f] : -1;
        const int64_t src = nb >= 0 ? (int64_t)nb : cid;
#pragma unroll
        for (int ec = 0; ec < 3; ++ec) fo[ec] = fn[(cid * 6 + f) * 3 * NF + tt + ec * NF];
        ho[0] = fh[(cid * 6 + f) * NF + tt];
        ho[1] = fh[(src * 6 + (nb >= 0 ? (f ^ 1) : f)) * NF + tt];
    };
    face_data(0, fnx, fhx);
    __builtin_amdgcn_sched_barrier(0);
    if (t < NF) sB[t] = fbv;
    if (act) {
#pragma unroll
        for (int ec = 0; ec < 3; ++ec)
#pragma unroll
            for (int u = 0; u < N; ++u) sU[lc][ec][tt + u * NF] = uv[ec][u];
    }
    __syncthreads();
    const LaneB<N> LB(sB, a, b);
    // interior faces first, while all three velocity layers are in LDS:
    // tau ds {hr u . n_K} at the Gauss points, back to the nodes; the
    // neighbour's face layers are gathered into LDS first
    double Yf[N];
#pragma unroll
    for (int i = 0; i < N; ++i) Yf[i] = 0.0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, s = f & 1;
        const int32_t nb = act ? nbr6[f] : -1;
        // this face's data, and the next face's requested now
        double fcur[3], hcur[2];
#pragma unroll
        for (int ec = 0; ec < 3; ++ec) fcur[ec] = fnx[ec];
        hcur[0] = fhx[0];
        hcur[1] = fhx[1];
        if (f < 5) face_data(f + 1, fnx, fhx);
        if (nb >= 0) {
#pragma unroll
            for (int ec = 0; ec < 3; ++ec) sL[lc][ec][tt] = nbu[f][ec];
        }
        __syncthreads();
        if (act) {
            double g = 0.0;
            if (nb >= 0) {
                double fo = 0.0, fnb = 0.0;
                for (int ec = 0; ec < 3; ++ec) {
                    const double uo = trace_at<N>(LB, sU[lc][ec], d, s ? N - 1 : 0);
                    const double un = trace_at2<N>(LB, sL[lc][ec]);
                    fo += uo * fcur[ec];
                    fnb += un * fcur[ec];
                }
                fo *= hcur[0];
                fnb *= hcur[1];
                g = tau * 0.5 * (fo + fnb);
            }
            sG[lc][tt] = g;
        }
        __syncthreads();
        if (act) sA[lc][tt] = trace_t<N>(LB, sG[lc]);
        __syncthreads();
        if (act) add_face<N>(sA[lc], f, a, b, Yf);
    }
    // cell terms: the velocity at the Gauss points, the weighted metric
    // terms, the transposed gradient; once at the Gauss points the second
    // and third velocity layers serve as its scratch
    double uq[3][N];
#pragma unroll
    for (int ec = 0; ec < 3; ++ec) to_gauss<N>(sU[lc][ec], sF[lc], act, a, b, uq[ec]);
    double t0[N], t1[N], t2[N], Y[N];
    if (act) {
        const double *Wc = WC + cid * 9 * ND + a + N * b;
        for (int q = 0; q < N; ++q) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int ec = 0; ec < 3; ++ec) {
                s0 += Wc[(0 + ec) * ND + NF * q] * uq[ec][q];
                s1 += Wc[(3 + ec) * ND + NF * q] * uq[ec][q];
                s2 += Wc[(6 + ec) * ND + NF * q] * uq[ec][q];
            }
            t0[q] = s0;
            t1[q] = s1;
            t2[q] = s2;
        }
    }
    grad_t<N>(sF[lc], sU[lc][1], sU[lc][2], act, a, b, t0, t1, t2, tau, Y);
    if (act)
#pragma unroll
        for (int i = 0; i < N; ++i) Y[i] += Yf[i];
    if (DP) {
        // D x: x at the Gauss points, times md, back to the nodes (x and md
        // requested together)
        double xl[N], mdq[N];
#pragma unroll
        for (int u = 0; u < N; ++u) {
            xl[u] = xv[cid * ND + tt + u * NF];
            mdq[u] = md[cid * ND + a + N * b + NF * u];
        }
        __builtin_amdgcn_sched_barrier(0);
        if (act) {
#pragma unroll
            for (int u = 0; u < N; ++u) sU[lc][0][tt + u * NF] = xl[u];
        }
        __syncthreads();
        double xq[N], dx[N];
        to_gauss<N>(sU[lc][0], sF[lc], act, a, b, xq);
        if (act)
#pragma unroll
            for (int q = 0; q < N; ++q) xq[q] *= mdq[q];
        interp_t<N>(sF[lc], act, a, b, xq, dx);
        if (act)
#pragma unroll
            for (int i = 0; i < N; ++i) Y[i] = dx[i] - Y[i];
    }
    if (act) {
        const int64_t o = cid * ND + N * a + NF * b;
        if (DP && bv)
            for (int i = 0; i < N; ++i) qv[o + i] = bv[o + i] - Y[i];
        else
            for (int i = 0; i < N; ++i) qv[o + i] = Y[i];
    }
}

template <int N>
hipError_t grad_n(hx_ctx *c, const double *p, double *u3, bool minv)
{
    const int cpb = PCfg<N, GRAD_T>::CPB;
    const int nb = (int)((c->n_cells + cpb - 1) / cpb);
    if (minv)
        hipLaunchKernelGGL((k_grad<N, true>), dim3(nb), dim3(PCfg<N, GRAD_T>::NT), 0, c->stream, p, u3,
                           c->n_dofs, c->psW, c->psFn, c->visitp, c->ref, c->ps_tau, (int)c->n_cells,
                           nb, c->psMr);
    else
        hipLaunchKernelGGL((k_grad<N, false>), dim3(nb), dim3(PCfg<N, GRAD_T>::NT), 0, c->stream, p,
                           u3, c->n_dofs, c->psW, c->psFn, c->visitp, c->ref, c->ps_tau,
                           (int)c->n_cells, nb, (const double *)nullptr);
    return hipGetLastError();
}

template <int N>
hipError_t div_n(hx_ctx *c, const double *u3, double *q, const double *x, const double *b)
{
    const int cpb = PCfg<N, DIV_T>::CPB;
    const int nb = (int)((c->n_cells + cpb - 1) / cpb);
    if (x)
        hipLaunchKernelGGL((k_div<N, true>), dim3(nb), dim3(PCfg<N, DIV_T>::NT), 0, c->stream, u3, q,
                           c->n_dofs, c->psWC, c->psFn, c->psFh, c->visitp, c->ref, c->ps_tau,
                           (int)c->n_cells, nb, x, c->psMd, b);
    else
        hipLaunchKernelGGL((k_div<N, false>), dim3(nb), dim3(PCfg<N, DIV_T>::NT), 0, c->stream, u3, q,
                           c->n_dofs, c->psWC, c->psFn, c->psFh, c->visitp, c->ref, c->ps_tau,
                           (int)c->n_cells, nb, (const double *)nullptr, (const double *)nullptr,
                           (const double *)nullptr);
    return hipGetLastError();
}

hipError_t grad_dispatch(hx_ctx *c, const double *p, double *u3, bool minv)
{
    switch (c->n) {
    case 2: return grad_n<2>(c, p, u3, minv);
    case 3: return grad_n<3>(c, p, u3, minv);
    case 4: return grad_n<4>(c, p, u3, minv);
    case 5: return grad_n<5>(c, p, u3, minv);
    case 6: return grad_n<6>(c, p, u3, minv);
    case 7: return grad_n<7>(c, p, u3, minv);
    case 8: return grad_n<8>(c, p, u3, minv);
    default: return hipErrorInvalidValue;
    }
}

hipError_t div_dispatch(hx_ctx *c, const double *u3, double *q, const double *x, const double *b)
{
    switch (c->n) {
    case 2: return div_n<2>(c, u3, q, x, b);
    case 3: return div_n<3>(c, u3, q, x, b);
    case 4: return div_n<4>(c, u3, q, x, b);
    case 5: return div_n<5>(c, u3, q, x, b);
    case 6: return div_n<6>(c, u3, q, x, b);
    case 7: return div_n<7>(c, u3, q, x, b);
    case 8: return div_n<8>(c, u3, q, x, b);
    default: return hipErrorInvalidValue;
    }
}

// h = gamma p / ((gamma - 1) rho): specific enthalpy of an ideal gas
__global__ void k_enthalpy(int64_t n, const double *__restrict__ p, const double *__restrict__ rho,
                           double f, double *h)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) h[i] = f * p[i] / rho[i];
}

}  // namespace

hipError_t launch_enthalpy(hx_ctx *c, const double *p, const double *rho, double gamma, double *h)
{
    const int64_t n = c->n_dofs;
    hipLaunchKernelGGL(k_enthalpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, p,
                       rho, gamma / (gamma - 1.0), h);
    return hipGetLastError();
}

hipError_t launch_grad(hx_ctx *c, const double *p, double *u3) { return grad_dispatch(c, p, u3, false); }

hipError_t launch_div(hx_ctx *c, const double *u3, double *q) { return div_dispatch(c, u3, q, nullptr, nullptr); }

// y = S x = D x - C A^-1 B x, or y = b - S x when b is given: two passes,
// v = A^-1 B x (the mass inverse in the gradient's epilogue), then
// D x - C v (the mass of x in the divergence's epilogue)
hipError_t press_apply64(hx_ctx *c, const double *x, double *y, const double *b)
{
    double *v3 = c->psWork + 3 * c->n_dofs;
    hipError_t e = grad_dispatch(c, x, v3, true);
    return e != hipSuccess ? e : div_dispatch(c, v3, y, x, b);
}

}  // namespace hx
