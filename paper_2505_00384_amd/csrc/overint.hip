// The operator with consistent integration (paper section 3.3: a Gauss rule
// of 2r+1 points per direction, which integrates the products of three
// polynomials of the variable-coefficient terms without aliasing, against
// the r+1 points of the fast evaluation).  Same form as k_apply; the 1-D
// interpolation B (nq x n) and its derivative BD are rectangular now, so the
// sweeps change pencil lengths (n nodes <-> nq points).
//
// One cell per block.  Cell part: x sweep by lanes (j, l) (n^2), y sweep by
// lanes (qx, l) (nq n), z sweep, quadrature-point operation and transposed z
// sweep by lanes (qx, qy) (nq^2), transposed y and x sweeps back; fields in
// LDS between the sweeps.  Face part, face by face: lanes (e1, e2) form the
// own and the neighbour's face layer and normal-derivative column (the
// derivative of the GLL basis at the face end), lanes (a, b) evaluate value,
// tangential and normal derivatives at the nq^2 face points and the flux
// terms, lanes (e1, e2) contract them back to layer weights, and the pencil
// owners add them (layer weights to the face layer, derivative weights
// along the normal lines).  One thread writes each output.
#include "common.hpp"

namespace hx {
namespace {

// compile-time B and BD at the 2N-1 Gauss points (generated at build time
// from the library's rules, the same values as the set-up tables)
template <int N> struct KBQ;
template <int N> struct KBDQ;
#include "optables_q.inc"

template <int N>
__device__ __forceinline__ constexpr double tq(int q, int i) { return KBQ<N>::d[q * N + i]; }
template <int N>
__device__ __forceinline__ constexpr double tdq(int q, int i) { return KBDQ<N>::d[q * N + i]; }

template <int N, int Q>
struct QCfg {
    static constexpr int ND = N * N * N, NF = N * N, Q2 = Q * Q, Q3 = Q * Q * Q;
    static constexpr int QN = Q * N, QNN = Q * N * N, QQN = Q * Q * N;
    static constexpr int NT = ((Q2 > QN ? Q2 : QN) + 63) / 64 * 64;
};

// threads per block for N nodes and 2N-1 points per direction
template <int N>
constexpr int q_nt() { return QCfg<N, 2 * N - 1>::NT; }

template <int N>
__device__ __forceinline__ int qlay(int d, int m, int e1, int e2)
{
    const int s1 = d == 0 ? N : 1, s2 = d == 2 ? N : N * N, sd = d == 0 ? 1 : (d == 1 ? N : N * N);
    return m * sd + e1 * s1 + e2 * s2;
}

template <int N>
__global__ void __launch_bounds__(q_nt<N>(), 4)
k_apply_q(const double *__restrict__ x, double *__restrict__ y, const double *__restrict__ cell,
          const double *__restrict__ face, const int32_t *__restrict__ nbr,
          const RefTabQ *__restrict__ TQ, const RefTab64 *__restrict__ T, int n_cells)
{
    constexpr int Q = 2 * N - 1;
    using C = QCfg<N, Q>;
    constexpr int ND = C::ND, NF = C::NF, Q2 = C::Q2, Q3 = C::Q3, QNN = C::QNN, QQN = C::QQN;
    __shared__ double sB[Q * N], sD[Q * N], sDL[2][N];
    __shared__ double sX[ND];
    __shared__ double FA[6][2][NF];
    // one pool for the sweep buffers of the cell part (U0, U1, V0, V1, V2)
    // and, once those are free, the face stage: U0 keeps the output pencils
    // and the face arrays overlay U1 .. V2
    // the face stage handles the two faces of one direction together: per
    // face 4 NF (layers), 6 QN (along e1), 4 Q2 (face points), 3 QN (back)
    constexpr int FACE1 = 4 * NF + 9 * C::QN + 4 * Q2;
    constexpr int CELLW = QNN + 3 * QQN, FACEW = 2 * FACE1;
    __shared__ double pool[QNN + (CELLW > FACEW ? CELLW : FACEW)];
    double *const U0 = pool, *const U1 = pool + QNN, *const V0 = U1 + QNN, *const V1 = V0 + QQN,
                 *const V2 = V1 + QQN;
    const int t = threadIdx.x;
    const int64_t cid = blockIdx.x;
    for (int e = t; e < Q * N; e += blockDim.x) {
        sB[e] = TQ->B[e];
        sD[e] = TQ->BD[e];
    }
    for (int e = t; e < 2 * N; e += blockDim.x) sDL[e / N][e % N] = T->DL[e / N][e % N];
    for (int e = t; e < ND; e += blockDim.x) sX[e] = x[cid * ND + e];
    __syncthreads();

    // x sweep: lane (j, l): u and du/dxi at (qx, j, l), layout qx + Q (j + N l)
    if (t < NF) {
        const int j = t % N, l = t / N;
        double v[N];
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = sX[i + N * j + NF * l];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int i = 0; i < N; ++i) {
                s0 += tq<N>(q, i) * v[i];
                s1 += tdq<N>(q, i) * v[i];
            }
            U0[q + Q * (j + N * l)] = s0;
            U1[q + Q * (j + N * l)] = s1;
        }
    }
    __syncthreads();
    // y sweep: lane (qx, l): u, d/deta (from u) and d/dxi (from U1) at
    // (qx, qy, l), layout qx + Q (qy + Q l)
    if (t < C::QN) {
        const int qx = t % Q, l = t / Q;
        double v0[N], v1[N];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            v0[j] = U0[qx + Q * (j + N * l)];
            v1[j] = U1[qx + Q * (j + N * l)];
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                s0 += tq<N>(q, j) * v0[j];
                s1 += tdq<N>(q, j) * v0[j];
                s2 += tq<N>(q, j) * v1[j];
            }
            V0[qx + Q * (q + Q * l)] = s0;
            V1[qx + Q * (q + Q * l)] = s1;
            V2[qx + Q * (q + Q * l)] = s2;
        }
    }
    __syncthreads();
    // z sweep, quadrature-point operation, transposed z sweep: lane (qx, qy)
    double w0[N], w1[N], w2[N];
    if (t < Q2) {
        const int qx = t % Q, qy = t / Q;
        double a0[N], a1[N], a2[N];
#pragma unroll
        for (int l = 0; l < N; ++l) {
            a0[l] = V0[qx + Q * (qy + Q * l)];
            a1[l] = V1[qx + Q * (qy + Q * l)];
            a2[l] = V2[qx + Q * (qy + Q * l)];
        }
#pragma unroll
        for (int l = 0; l < N; ++l) w0[l] = w1[l] = w2[l] = 0.0;
        const double *cp = cell + cid * 7 * Q3 + qx + Q * qy;
        // the point data of plane q + 1 are requested before plane q's
        // arithmetic, so one plane's loads are always in flight
        double nx[7];
#pragma unroll
        for (int k = 0; k < 7; ++k) nx[k] = cp[k * Q3];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double cd[7];
#pragma unroll
            for (int k = 0; k < 7; ++k) cd[k] = nx[k];
            if (q + 1 < Q) {
#pragma unroll
                for (int k = 0; k < 7; ++k) nx[k] = cp[Q2 * (q + 1) + k * Q3];
            }
            double u = 0.0, dz = 0.0, dy = 0.0, dx = 0.0;
#pragma unroll
            for (int l = 0; l < N; ++l) {
                u += tq<N>(q, l) * a0[l];
                dz += tdq<N>(q, l) * a0[l];
                dy += tq<N>(q, l) * a1[l];
                dx += tq<N>(q, l) * a2[l];
            }
            const double m = cd[0], gxx = cd[1], gxy = cd[2], gxz = cd[3], gyy = cd[4], gyz = cd[5],
                         gzz = cd[6];
            const double v = m * u;
            const double fx = gxx * dx + gxy * dy + gxz * dz;
            const double fy = gxy * dx + gyy * dy + gyz * dz;
            const double fz = gxz * dx + gyz * dy + gzz * dz;
#pragma unroll
            for (int l = 0; l < N; ++l) {
                w0[l] += tq<N>(q, l) * v + tdq<N>(q, l) * fz;
                w1[l] += tq<N>(q, l) * fy;
                w2[l] += tq<N>(q, l) * fx;
            }
        }
    }
    __syncthreads();
    if (t < Q2) {
        const int qx = t % Q, qy = t / Q;
        for (int l = 0; l < N; ++l) {
            V0[qx + Q * (qy + Q * l)] = w0[l];
            V1[qx + Q * (qy + Q * l)] = w1[l];
            V2[qx + Q * (qy + Q * l)] = w2[l];
        }
    }
    __syncthreads();
    // transposed y sweep: lane (qx, l) -> (qx, j, l): s0 = B^T w0 + BD^T w1,
    // s1 = B^T w2
    if (t < C::QN) {
        const int qx = t % Q, l = t / Q;
        double s0[N], s1[N];
#pragma unroll
        for (int j = 0; j < N; ++j) s0[j] = s1[j] = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double a0 = V0[qx + Q * (q + Q * l)], a1 = V1[qx + Q * (q + Q * l)],
                         a2 = V2[qx + Q * (q + Q * l)];
#pragma unroll
            for (int j = 0; j < N; ++j) {
                s0[j] += tq<N>(q, j) * a0 + tdq<N>(q, j) * a1;
                s1[j] += tq<N>(q, j) * a2;
            }
        }
        for (int j = 0; j < N; ++j) {
            U0[qx + Q * (j + N * l)] = s0[j];
            U1[qx + Q * (j + N * l)] = s1[j];
        }
    }
    __syncthreads();
    // transposed x sweep: lane (j, l) keeps its output pencil
    double Y[N];
    if (t < NF) {
        const int j = t % N, l = t / N;
#pragma unroll
        for (int i = 0; i < N; ++i) Y[i] = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const double a0 = U0[q + Q * (j + N * l)], a1 = U1[q + Q * (j + N * l)];
#pragma unroll
            for (int i = 0; i < N; ++i) Y[i] += tq<N>(q, i) * a0 + tdq<N>(q, i) * a1;
        }
    }

    // ---------------------------------------------------------------- faces
    // The output pencils wait in LDS (U0, free after the transposed x
    // sweep) while the faces run, the two faces of each direction together.
    // Per face, sum-factorised in two 1-D steps each way: items (e1, e2)
    // form the own and the neighbour's face layer and normal-derivative
    // column; items (a, e2) contract along e1 (value and e1-derivative of
    // both layers, value of both derivative columns); items (a, b) contract
    // along e2 and form the flux terms at the face points; items (e1, b) and
    // then (e1, e2) contract back.
    __syncthreads();
    double *sY = U0;
    if (t < NF) {
        const int j = t % N, l = t / N;
#pragma unroll
        for (int i = 0; i < N; ++i) sY[i + N * j + NF * l] = Y[i];
    }
    for (int d = 0; d < 3; ++d) {
        const int32_t nbs[2] = {nbr[6 * cid + 2 * d], nbr[6 * cid + 2 * d + 1]};
        // layers and normal-derivative columns of face (d, s), own and
        // neighbour side: item (s, e1, e2)
        for (int it = t; it < 2 * NF; it += blockDim.x) {
            const int s = it / NF, k = it - s * NF;
            const int32_t nb = nbs[s];
            if (nb < 0) {
                FA[2 * d + s][0][k] = FA[2 * d + s][1][k] = 0.0;
                continue;
            }
            double *F = U1 + s * FACE1;
            const int e1 = k % N, e2 = k / N;
            const int mo = s ? N - 1 : 0, mn = s ? 0 : N - 1;
            const double *xn = x + (int64_t)nb * ND;
            double dov = 0.0, dnv = 0.0;
            for (int m = 0; m < N; ++m) {
                dov += sDL[s][m] * sX[qlay<N>(d, m, e1, e2)];
                dnv += sDL[1 - s][m] * xn[qlay<N>(d, m, e1, e2)];
            }
            F[k] = sX[qlay<N>(d, mo, e1, e2)];
            F[NF + k] = dov;
            F[2 * NF + k] = xn[qlay<N>(d, mn, e1, e2)];
            F[3 * NF + k] = dnv;
        }
        __syncthreads();
        // along e1: item (s, a, e2)
        for (int it = t; it < 2 * C::QN; it += blockDim.x) {
            const int s = it / C::QN, k = it - s * C::QN;
            if (nbs[s] < 0) continue;
            const double *F = U1 + s * FACE1;
            double *Tf = U1 + s * FACE1 + 4 * NF;
            const int a = k % Q, e2 = k / Q;
            double c0 = 0, c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0;
#pragma unroll
            for (int e1 = 0; e1 < N; ++e1) {
                const double ba = sB[a * N + e1], da = sD[a * N + e1];
                const int kk = e1 + N * e2;
                c0 += ba * F[kk];
                c1 += da * F[kk];
                c2 += ba * F[NF + kk];
                c3 += ba * F[2 * NF + kk];
                c4 += da * F[2 * NF + kk];
                c5 += ba * F[3 * NF + kk];
            }
            Tf[0 * C::QN + k] = c0;
            Tf[1 * C::QN + k] = c1;
            Tf[2 * C::QN + k] = c2;
            Tf[3 * C::QN + k] = c3;
            Tf[4 * C::QN + k] = c4;
            Tf[5 * C::QN + k] = c5;
        }
        __syncthreads();
        // along e2 and the flux terms: item (s, a, b)
        for (int it = t; it < 2 * Q2; it += blockDim.x) {
            const int s = it / Q2, k = it - s * Q2;
            const int32_t nb = nbs[s];
            if (nb < 0) continue;
            const double *Tf = U1 + s * FACE1 + 4 * NF;
            double *P = U1 + s * FACE1 + 4 * NF + 6 * C::QN;
            const int a = k % Q, b = k / Q;
            double vo = 0, t1o = 0, t2o = 0, dno = 0, vn = 0, t1n = 0, t2n = 0, dnn = 0;
#pragma unroll
            for (int e2 = 0; e2 < N; ++e2) {
                const double bb = sB[b * N + e2], db = sD[b * N + e2];
                const int kk = a + Q * e2;
                vo += bb * Tf[0 * C::QN + kk];
                t1o += bb * Tf[1 * C::QN + kk];
                t2o += db * Tf[0 * C::QN + kk];
                dno += bb * Tf[2 * C::QN + kk];
                vn += bb * Tf[3 * C::QN + kk];
                t1n += bb * Tf[4 * C::QN + kk];
                t2n += db * Tf[3 * C::QN + kk];
                dnn += bb * Tf[5 * C::QN + kk];
            }
            const int64_t fid = s ? cid : (int64_t)nb;
            const double *fd = face + (fid * 3 + d) * 7 * Q2 + k;
            const int go = s ? 0 : 3, gn = s ? 3 : 0;
            const double flux = fd[go * Q2] * dno + fd[(go + 1) * Q2] * t1o + fd[(go + 2) * Q2] * t2o +
                                fd[gn * Q2] * dnn + fd[(gn + 1) * Q2] * t1n + fd[(gn + 2) * Q2] * t2n;
            const double jump = s ? (vo - vn) : (vn - vo);
            const double sg = s ? 1.0 : -1.0;
            const double hj = -0.5 * jump;
            P[k] = sg * (-0.5 * flux + fd[6 * Q2] * jump);            // value weight
            P[Q2 + k] = hj * fd[(go + 1) * Q2];                       // e1-derivative weight
            P[2 * Q2 + k] = hj * fd[(go + 2) * Q2];                   // e2-derivative weight
            P[3 * Q2 + k] = hj * fd[go * Q2];                         // normal-derivative weight
        }
        __syncthreads();
        // back along a: item (s, e1, b)
        for (int it = t; it < 2 * C::QN; it += blockDim.x) {
            const int s = it / C::QN, k = it - s * C::QN;
            if (nbs[s] < 0) continue;
            const double *P = U1 + s * FACE1 + 4 * NF + 6 * C::QN;
            double *Gf = U1 + s * FACE1 + 4 * NF + 6 * C::QN + 4 * Q2;
            const int e1 = k % N, b = k / N;
            double g = 0, h = 0, kk = 0;
#pragma unroll
            for (int a = 0; a < Q; ++a) {
                const double ba = sB[a * N + e1], da = sD[a * N + e1];
                const int pk = a + Q * b;
                g += ba * P[pk] + da * P[Q2 + pk];
                h += ba * P[2 * Q2 + pk];
                kk += ba * P[3 * Q2 + pk];
            }
            Gf[0 * C::QN + k] = g;
            Gf[1 * C::QN + k] = h;
            Gf[2 * C::QN + k] = kk;
        }
        __syncthreads();
        // back along b: item (s, e1, e2)
        for (int it = t; it < 2 * NF; it += blockDim.x) {
            const int s = it / NF, k = it - s * NF;
            if (nbs[s] < 0) continue;
            const double *Gf = U1 + s * FACE1 + 4 * NF + 6 * C::QN + 4 * Q2;
            const int e1 = k % N, e2 = k / N;
            double f0 = 0.0, f1 = 0.0;
#pragma unroll
            for (int b = 0; b < Q; ++b) {
                const double bb = sB[b * N + e2], db = sD[b * N + e2];
                const int gk = e1 + N * b;
                f0 += bb * Gf[0 * C::QN + gk] + db * Gf[1 * C::QN + gk];
                f1 += bb * Gf[2 * C::QN + gk];
            }
            FA[2 * d + s][0][k] = f0;
            FA[2 * d + s][1][k] = f1;
        }
        __syncthreads();
    }
    __syncthreads();
    // pencil owners (j, l) add the six faces
    if (t < NF) {
        const int j = t % N, l = t / N;
        double Yp[N];
#pragma unroll
        for (int i = 0; i < N; ++i) Yp[i] = sY[i + N * j + NF * l];
        for (int s = 0; s < 2; ++s) {
            const int layer = s ? N - 1 : 0;
            // x faces: normal coordinate i, (e1, e2) = (j, l)
            {
                const double f0 = FA[s][0][j + N * l], f1 = FA[s][1][j + N * l];
                for (int i = 0; i < N; ++i) Yp[i] += sDL[s][i] * f1 + (i == layer ? f0 : 0.0);
            }
            // y faces: normal coordinate j, (e1, e2) = (i, l)
            for (int i = 0; i < N; ++i)
                Yp[i] += sDL[s][j] * FA[2 + s][1][i + N * l] + (j == layer ? FA[2 + s][0][i + N * l] : 0.0);
            // z faces: normal coordinate l, (e1, e2) = (i, j)
            for (int i = 0; i < N; ++i)
                Yp[i] += sDL[s][l] * FA[4 + s][1][i + N * j] + (l == layer ? FA[4 + s][0][i + N * j] : 0.0);
        }
        for (int i = 0; i < N; ++i) y[cid * ND + i + N * j + NF * l] = Yp[i];
    }
}

template <int N>
hipError_t apply_q_n(hx_ctx *c, const double *x, double *y)
{
    constexpr int Q = 2 * N - 1;
    hipLaunchKernelGGL(k_apply_q<N>, dim3((unsigned)c->n_cells), dim3(QCfg<N, Q>::NT), 0,
                       c->stream, x, y, c->qcell, c->qface, c->nbr, c->refq, c->ref, (int)c->n_cells);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_apply_q(hx_ctx *c, const double *x, double *y)
{
    if (c->nq != 2 * c->n - 1) return hipErrorInvalidValue;
    switch (c->n) {
    case 2: return apply_q_n<2>(c, x, y);
    case 3: return apply_q_n<3>(c, x, y);
    case 4: return apply_q_n<4>(c, x, y);
    case 5: return apply_q_n<5>(c, x, y);
    case 6: return apply_q_n<6>(c, x, y);
    case 7: return apply_q_n<7>(c, x, y);
    case 8: return apply_q_n<8>(c, x, y);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hx
