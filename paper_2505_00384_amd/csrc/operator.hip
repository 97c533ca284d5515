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
//    transpose returns to columns for the last transposed sweep.  The two
//    sides pass through the same three fields of LDS one after the other, and
//    the transposed sweeps write over what they read, so a face needs 3 N^2
//    values of LDS.  The
//    pencil owners then add the six faces' layer and normal-derivative
//    contributions to their own output values.  Each output value is written
//    by exactly one lane (no atomics; bitwise reproducible).
//  * the 1-D tables are compile-time constants and loops over them are
//    unrolled, so their entries are wave-uniform scalar operands.
//  * cell data [cell][7][N^3] is streamed once with non-temporal loads; x and
//    the face data [cell][3][7][N][N] are read by neighbours too and stay
//    cacheable.
//  * affine cells (constant Jacobian) read compressed data instead: alpha w
//    detJ and beta w detJ at the points [cell][2][N^3] plus J^-1 J^-T once per
//    cell, and faces between two affine cells read beta- w, beta+ w per point
//    [cell][3][2][N][N] plus seven constants per face; the last word of the
//    traversal record says which cell and faces are compressed (one bit each),
//    so no extra round trip decides it.  The merged values are rebuilt in
//    registers where they are used (m = a, G = b J^-1 J^-T; g = (beta w) v,
//    s = sd ((beta- w) + (beta+ w))).
//  * cells are visited in the order of a host-built permutation (one 32-byte
//    record per slot holds the cell and its six neighbours): tiles of
//    columns swept layer by layer, in one contiguous range per XCD, so the
//    neighbours a cell reads were touched recently by the same XCD's L2.
#include "common.hpp"

#include <type_traits>

namespace hx {

namespace {

// compile-time copies of the 1-D tables (generated at build time from the
// library's rules): with every loop unrolled the compiler materialises the
// entries as scalar operands instead of loading them
template <int N> struct KB;
template <int N> struct KBD;
template <int N> struct KDL;
#include "optables.inc"

template <typename T, int N>
__device__ __forceinline__ T tE(int e, int i)
{
    if constexpr (std::is_same<T, double>::value) return KDL<N>::d[e * N + i];
    else return KDL<N>::f[e * N + i];
}

// ---------------------------------------------------------------------------
// Even-odd evaluation of the 1-D contractions.  Gauss points and GLL nodes lie
// symmetric about the centre, so B(N-1-q, N-1-i) = B(q, i) and
// BD(N-1-q, N-1-i) = -BD(q, i), and the same holds for the transposes.  With
// a pencil split into e_i = u_i + u_{N-1-i}, o_i = u_i - u_{N-1-i} (i < N/2)
// and the middle value (N odd), rows r and N-1-r of a contraction come out as
// the sum and difference of two partial sums over N/2 terms each, which
// removes about a quarter of the multiply-adds for N = 5.

// entry (r, c) of B (W = 0) or BD (W = 1), or of its transpose (TR)
template <int N, int W, bool TR>
__device__ __forceinline__ double tab(int r, int c)
{
    const int q = TR ? c : r, i = TR ? r : c;
    return W ? KBD<N>::d[q * N + i] : KB<N>::d[q * N + i];
}

// split of a pencil into its even and odd parts
template <typename T, int N>
struct EvenOdd {
    static constexpr int H = N / 2;
    T e[H], o[H], m;
    __device__ __forceinline__ explicit EvenOdd(const T (&u)[N])
    {
#pragma unroll
        for (int i = 0; i < H; ++i) {
            e[i] = u[i] + u[N - 1 - i];
            o[i] = u[i] - u[N - 1 - i];
        }
        m = (N & 1) ? u[H] : T(0);
    }
};

// output pencil as mirror-even (P) and mirror-odd (Q) partial sums of its
// first (N+1)/2 rows: y_r = P_r + Q_r, y_{N-1-r} = P_r - Q_r
template <typename T, int N>
struct Rows {
    static constexpr int H = N / 2, R = (N + 1) / 2;
    T P[R], Q[R];
    __device__ __forceinline__ Rows()
    {
#pragma unroll
        for (int r = 0; r < R; ++r) P[r] = Q[r] = T(0);
    }
    // add M x with M = B or BD (W) or a transpose (TR); for a symmetric M the
    // even part of x feeds P and the odd part Q, for an antisymmetric M the
    // other way round; in the middle row (N odd) the part that vanishes by
    // symmetry is skipped
    template <int W, bool TR>
    __device__ __forceinline__ void add(const EvenOdd<T, N> &x)
    {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const bool mid = (N & 1) && r == H;
            T &pe = W ? Q[r] : P[r];   // receives the even part
            T &po = W ? P[r] : Q[r];   // receives the odd part
            if (!(W && mid)) {
                if (N & 1) pe += T(tab<N, W, TR>(r, H)) * x.m;
#pragma unroll
                for (int i = 0; i < H; ++i)
                    pe += T(0.5 * (tab<N, W, TR>(r, i) + tab<N, W, TR>(r, N - 1 - i))) * x.e[i];
            }
            if (!(!W && mid)) {
#pragma unroll
                for (int i = 0; i < H; ++i)
                    po += T(0.5 * (tab<N, W, TR>(r, i) - tab<N, W, TR>(r, N - 1 - i))) * x.o[i];
            }
        }
    }
    __device__ __forceinline__ void out(T (&y)[N]) const
    {
#pragma unroll
        for (int r = 0; r < H; ++r) {
            y[r] = P[r] + Q[r];
            y[N - 1 - r] = P[r] - Q[r];
        }
        if (N & 1) y[H] = P[H];
    }
};

// y = B u (W = 0) or BD u (W = 1) along a pencil; transposed with TR
template <typename T, int N, int W, bool TR>
__device__ __forceinline__ void contract(const EvenOdd<T, N> &x, T (&y)[N])
{
    Rows<T, N> acc;
    acc.template add<W, TR>(x);
    acc.out(y);
}
// y = B^T u + BD^T v
template <typename T, int N>
__device__ __forceinline__ void contract_t2(const T (&u)[N], const T (&v)[N], T (&y)[N])
{
    Rows<T, N> acc;
    acc.template add<0, true>(EvenOdd<T, N>(u));
    acc.template add<1, true>(EvenOdd<T, N>(v));
    acc.out(y);
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
    static constexpr int GS = (18 * NF > 3 * ND) ? 18 * NF : 3 * ND;  // work area per cell
    static_assert(NF <= 64 && 6 * N <= 64, "one wave per cell at most");
};

// waves per SIMD the register budget is sized for (measured at N = 5 FP64:
// 2 waves with 160 registers is as fast as 3 and much faster than 4, which
// spills; the memory pipeline, not occupancy, sets the pace)
template <int N, typename T>
struct Occ {
    static constexpr int W = sizeof(T) == 8 ? (N <= 3 ? 4 : (N <= 4 ? 3 : 2))
                                            : (N <= 4 ? 4 : (N <= 6 ? 3 : 2));
    // the launch of affine cells keeps fewer values in registers (2 instead
    // of 7 per point), so it fits one more wave per SIMD without spilling
    // (measured at N = 5 FP64: 2.98 -> 2.83 ms for the whole operator on the
    // 256x64x64 channel, 45 % of its cells affine)
    static constexpr int WA = sizeof(T) == 8 ? (N <= 3 ? 4 : (N <= 5 ? 3 : 2)) : (N <= 7 ? 4 : 3);
    // request the quadrature-point data before the y sweep (register cost 7 N)
    static constexpr bool PREFETCH_CELL = N <= 5;
};

template <typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    return __builtin_nontemporal_load(p);
}

// PART: 0 the whole operator, 1 the cell integrals only, 2 the face terms only;
// AFF: the wave serves affine cells (compressed cell data; faces compressed
// where the record's mask says so) or general cells (general data only)
template <int N, typename T, bool DOT, int PART, bool AFF>
__device__ __forceinline__ void apply_body(
    const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ bvec,
    const T *__restrict__ cell, const T *__restrict__ face, const T *__restrict__ acell,
    const T *__restrict__ kk, const T *__restrict__ aface, const T *__restrict__ fcon,
    const int32_t *__restrict__ visit, int n_cells, int wg, int bid, double *__restrict__ dpart,
    T (&sU)[Cfg<N>::CPW][Cfg<N>::ND], T (&sG)[Cfg<N>::CPW][Cfg<N>::GS],
    T (&sXd)[DOT ? Cfg<N>::CPW : 1][DOT ? Cfg<N>::ND : 1])
{
    constexpr bool DO_CELL = PART != 2, DO_FACE = PART != 1;
    constexpr int NF = Cfg<N>::NF, ND = Cfg<N>::ND, LPC = Cfg<N>::LPC, CPW = Cfg<N>::CPW;

    const int lane = threadIdx.x;
    const int cs = lane / LPC;             // cell slot in the wave
    const int ln = lane - cs * LPC;        // lane within the cell
    const int slot = wg * CPW + cs;
    // the slot's record {cell, neighbours -x,+x,-y,+y,-z,+z, mask}: one
    // 32-byte line gives every index this wave needs; a record whose cell is
    // -1 pads a group of records to whole waves
    const int32_t *rec = visit + (int64_t)(slot < n_cells ? slot : 0) * 8;
    const int32_t rc = rec[0];
    const bool valid = slot < n_cells && rc >= 0;
    const int64_t cid = valid ? rc : 0;
    // bit 1 + f of the record's last word: face f is read compressed
    const int32_t cmask = (AFF && valid) ? rec[7] : 0;
    constexpr bool caff = AFF;
    T *G = &sG[cs][0];
    T *U = &sU[cs][0];

    // ---- cell lanes: (a, b), pencil owners
    const bool cl = valid && ln < NF;
    const int a = ln % N, b = (ln / N) % N;
    // ---- face lanes: (f, p), column owners
    const bool fl0 = valid && ln < 6 * N;
    const int f = fl0 ? ln / N : 0, rr = ln % N;
    const int d = f >> 1, s = f & 1;
    const int32_t nb = (DO_FACE && fl0) ? rec[1 + f] : -1;
    const bool fl = nb >= 0;
    const bool fcmp = AFF && ((cmask >> (1 + f)) & 1);
    // strides of the normal index m, the column index p and the row index r
    // of the face's direction in a cell's lexicographic numbering
    const int sm = d == 0 ? 1 : (d == 1 ? N : NF);
    const int sp = d == 0 ? N : 1;
    const int sr = d == 2 ? N : NF;

    // own values: all loads first, then the LDS stores
    constexpr int XL = (ND + LPC - 1) / LPC;
    T xv[XL];
#pragma unroll
    for (int k = 0; k < XL; ++k) {
        const int e = ln + k * LPC;
        xv[k] = (valid && e < ND) ? x[cid * ND + e] : T(0);
    }

    // The neighbour's layer values and normal derivatives on column p of
    // face f, loaded with the own values so that both arrive in one memory
    // round trip; the N lanes of a face read neighbouring addresses.  The
    // normal line is walked from the shared face inwards, so both sides use
    // the derivative weights of the lower end: for symmetric nodes the
    // weights at the upper end are those of the lower end mirrored and
    // negated.
    T Ln[N], Nn[N];
    if (fl) {
        // the neighbour touches with its upper layer when s = 0
        const int m0 = s ? 0 : (N - 1) * sm, dm = s ? sm : -sm;
        const T sgn = s ? T(1) : T(-1);
        const T *xn = x + (int64_t)nb * ND + rr * sp + m0;
#pragma unroll
        for (int r = 0; r < N; ++r) {
            T sn = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) sn += tE<T, N>(0, m) * xn[r * sr + m * dm];
            Nn[r] = sgn * sn;
            Ln[r] = xn[r * sr];
        }
    }
#pragma unroll
    for (int k = 0; k < XL; ++k) {
        const int e = ln + k * LPC;
        if (valid && e < ND) {
            U[e] = xv[k];
            if constexpr (DOT) sXd[cs][e] = xv[k];   // kept for x.(A x)
        }
    }

    // quadrature-point data of this lane's z pencil, streamed once: the
    // seven merged values, or for an affine cell alpha w detJ and beta w detJ
    // (in cdat[0] and cdat[1]) and J^-1 J^-T of the cell
    const T *cp = caff ? acell + cid * 2 * ND + a + N * b : cell + cid * 7 * ND + a + N * b;
    T kq[6];
    if (DO_CELL && cl && caff) {
#pragma unroll
        for (int s2 = 0; s2 < 6; ++s2) kq[s2] = kk[cid * 8 + s2];
    }
    __syncthreads();

    T Y[N];
    // =========================================================== cell part
    // x sweep: lane (j=a, l=b): B u and BD u along x
    if constexpr (!DO_CELL) {
#pragma unroll
        for (int i = 0; i < N; ++i) Y[i] = T(0);
    }
    if constexpr (DO_CELL) {
    if (cl) {
        T r[N], s0[N], s1[N];
#pragma unroll
        for (int i = 0; i < N; ++i) r[i] = U[i + N * a + NF * b];
        const EvenOdd<T, N> xr(r);
        contract<T, N, 0, false>(xr, s0);
        contract<T, N, 1, false>(xr, s1);
#pragma unroll
        for (int q = 0; q < N; ++q) {
            G[q + N * a + NF * b] = s0[q];
            G[ND + q + N * a + NF * b] = s1[q];
        }
    }
    __syncthreads();
    // quadrature-point data, requested before the y sweep so that the
    // stream is in flight while it runs
    T cdat[7][N];
    if (DO_CELL && Occ<N, T>::PREFETCH_CELL && cl) {
        if (caff) {
#pragma unroll
            for (int q = 0; q < N; ++q)
#pragma unroll
                for (int k = 0; k < 2; ++k) cdat[k][q] = ld_stream(cp + NF * q + k * ND);
        } else {
#pragma unroll
            for (int q = 0; q < N; ++q)
#pragma unroll
                for (int k = 0; k < 7; ++k) cdat[k][q] = ld_stream(cp + NF * q + k * ND);
        }
    }
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
            const EvenOdd<T, N> x0(p0), x1(p1);
            contract<T, N, 0, false>(x0, c0);
            contract<T, N, 1, false>(x0, c1);
            contract<T, N, 0, false>(x1, c2);
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
            }
            T uq[N], dzq[N], dyq[N], dxq[N];
            {
                const EvenOdd<T, N> x0(p0);
                contract<T, N, 0, false>(x0, uq);
                contract<T, N, 1, false>(x0, dzq);
                contract<T, N, 0, false>(EvenOdd<T, N>(p1), dyq);
                contract<T, N, 0, false>(EvenOdd<T, N>(p2), dxq);
            }
            T vq[N], fxq[N], fyq[N], fzq[N];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                const T u = uq[q], dz = dzq[q], dy = dyq[q], dx = dxq[q];
                T cq[7];
                if (Occ<N, T>::PREFETCH_CELL) {
#pragma unroll
                    for (int k = 0; k < 7; ++k) cq[k] = cdat[k][q];
                } else if (caff) {
#pragma unroll
                    for (int k = 0; k < 2; ++k) cq[k] = ld_stream(cp + NF * q + k * ND);
                } else {
#pragma unroll
                    for (int k = 0; k < 7; ++k) cq[k] = ld_stream(cp + NF * q + k * ND);
                }
                if (caff) {
                    const T bw = cq[1];
#pragma unroll
                    for (int k = 0; k < 6; ++k) cq[1 + k] = bw * kq[k];
                }
                const T m = cq[0], gxx = cq[1], gxy = cq[2], gxz = cq[3], gyy = cq[4], gyz = cq[5],
                        gzz = cq[6];
                vq[q] = m * u;
                fxq[q] = gxx * dx + gxy * dy + gxz * dz;
                fyq[q] = gxy * dx + gyy * dy + gyz * dz;
                fzq[q] = gxz * dx + gyz * dy + gzz * dz;
            }
            contract_t2<T, N>(vq, fzq, t0);
            contract<T, N, 0, true>(EvenOdd<T, N>(fyq), t1);
            contract<T, N, 0, true>(EvenOdd<T, N>(fxq), t2);
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
            contract_t2<T, N>(p0, p1, s0v);
            contract<T, N, 0, true>(EvenOdd<T, N>(p2), s1v);
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
        contract_t2<T, N>(p0, p1, Y);
    }
    __syncthreads();
    }   // DO_CELL

    // =========================================================== face part
    if constexpr (DO_FACE) {
    // The work area of a face holds three N x N fields at a time, laid out
    // [field][q2 or r][p].  Layer values and normal derivatives of a side are
    // interpolated along the second tangential direction by the column lanes
    // (f, p) (step 1), then along the first one by the row lanes (f, q2)
    // (step 2).  The neighbour side goes first and leaves its flux and value
    // at the row's Gauss points in registers; the own side then forms the
    // pointwise terms, sweeps back along the first direction in place (step
    // 3) and the column lanes finish the transposed sweep in place (step 4).
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    T *gf = G + f * 3 * NF;
    // step 1 of one side: fields B L, BD L, B Nd along the second direction
    auto interp_t2 = [&](const T (&L)[N], const T (&Nd)[N]) {
        T g0[N], g1[N], g2[N];
        const EvenOdd<T, N> xl(L);
        contract<T, N, 0, false>(xl, g0);
        contract<T, N, 1, false>(xl, g1);
        contract<T, N, 0, false>(EvenOdd<T, N>(Nd), g2);
#pragma unroll
        for (int q = 0; q < N; ++q) {
            gf[q * N + rr] = g0[q];
            gf[NF + q * N + rr] = g1[q];
            gf[2 * NF + q * N + rr] = g2[q];
        }
    };
    // face data of this row: [comp][q1][q2], components g-(3), g+(3), s
    const int64_t fid = s ? cid : (int64_t)nb;
    const T *fd = face + (fid * 3 + d) * 7 * NF + rr;
    // g of the neighbour side: g+ if the own cell is the minus cell
    const int gn_off = s ? 3 : 0, go_off = s ? 0 : 3;

    // face data of this row, all requested at once: g of the neighbour side,
    // g of the own side and the penalty factor at the row's N points; on a
    // compressed face beta w of the neighbour side (in gnb[0]) and of the own
    // side (in gow[0]) and the face's constants v-, v+, sd (in fcv)
    T gnb[3][N], gow[3][N], pn[N], fcv[7];
    if (fl) {
        if (fcmp) {
            const T *af = aface + (fid * 3 + d) * 2 * NF + rr;
            const int bn_off = s ? NF : 0, bo_off = s ? 0 : NF;
#pragma unroll
            for (int q1 = 0; q1 < N; ++q1) {
                gnb[0][q1] = af[bn_off + N * q1];
                gow[0][q1] = af[bo_off + N * q1];
            }
            const T *fp = fcon + (fid * 3 + d) * 8;
#pragma unroll
            for (int k = 0; k < 7; ++k) fcv[k] = fp[k];
        } else {
#pragma unroll
            for (int q1 = 0; q1 < N; ++q1) {
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    gnb[k][q1] = fd[(gn_off + k) * NF + N * q1];
                    gow[k][q1] = fd[(go_off + k) * NF + N * q1];
                }
                pn[q1] = fd[6 * NF + N * q1];
            }
        }
    }
    if (fl) interp_t2(Ln, Nn);
    __syncthreads();
    // step 2, neighbour side, lane (f, q2): flux and value at (q1, q2)
    T fnb[N], vnb[N];
    if (fl) {
        T h0[N], h1[N], h2[N];
#pragma unroll
        for (int p = 0; p < N; ++p) {
            h0[p] = gf[rr * N + p];
            h1[p] = gf[NF + rr * N + p];
            h2[p] = gf[2 * NF + rr * N + p];
        }
        T t1n[N], t2n[N], dnn[N];
        {
            const EvenOdd<T, N> x0(h0);
            contract<T, N, 0, false>(x0, vnb);
            contract<T, N, 1, false>(x0, t1n);
            contract<T, N, 0, false>(EvenOdd<T, N>(h1), t2n);
            contract<T, N, 0, false>(EvenOdd<T, N>(h2), dnn);
        }
        if (fcmp) {
            // v of the neighbour side: v+ if the own cell is the minus cell
            const T v0 = s ? fcv[3] : fcv[0], v1 = s ? fcv[4] : fcv[1], v2 = s ? fcv[5] : fcv[2];
#pragma unroll
            for (int q1 = 0; q1 < N; ++q1)
                fnb[q1] = gnb[0][q1] * (v0 * dnn[q1] + v1 * t1n[q1] + v2 * t2n[q1]);
        } else {
#pragma unroll
            for (int q1 = 0; q1 < N; ++q1)
                fnb[q1] = gnb[0][q1] * dnn[q1] + gnb[1][q1] * t1n[q1] + gnb[2][q1] * t2n[q1];
        }
    }
    __syncthreads();
    // step 1, own side, lane (f, p): layer and normal derivative from the
    // values in LDS
    if (fl) {
        // the own cell touches with its upper layer when s = 1
        const int m0 = s ? (N - 1) * sm : 0, dm = s ? -sm : sm;
        const T sgn = s ? T(-1) : T(1);
        const T *uo = U + rr * sp + m0;
        T Lo[N], No[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            T so = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) so += tE<T, N>(0, m) * uo[r * sr + m * dm];
            No[r] = sgn * so;
            Lo[r] = uo[r * sr];
        }
        interp_t2(Lo, No);
    }
    __syncthreads();
    // the own values are no longer needed: the output pencils wait in sU
    if (cl) {
#pragma unroll
        for (int i = 0; i < N; ++i) sU[cs][i + N * a + NF * b] = Y[i];
    }
    // steps 2 and 3, own side, lane (f, q2): pointwise terms and the
    // transposed sweep along the first direction, written over the row read
    if (fl) {
        T h0[N], h1[N], h2[N], A0[N], A1[N], A2[N];
#pragma unroll
        for (int p = 0; p < N; ++p) {
            h0[p] = gf[rr * N + p];
            h1[p] = gf[NF + rr * N + p];
            h2[p] = gf[2 * NF + rr * N + p];
        }
        T voq[N], t1q[N], t2q[N], dnq[N];
        {
            const EvenOdd<T, N> x0(h0);
            contract<T, N, 0, false>(x0, voq);
            contract<T, N, 1, false>(x0, t1q);
            contract<T, N, 0, false>(EvenOdd<T, N>(h1), t2q);
            contract<T, N, 0, false>(EvenOdd<T, N>(h2), dnq);
        }
        T cvq[N], ct1q[N], ct2q[N], cnq[N];
        // v of the own side (compressed face)
        T w0 = T(0), w1 = T(0), w2 = T(0);
        if (fcmp) {
            w0 = s ? fcv[0] : fcv[3];
            w1 = s ? fcv[1] : fcv[4];
            w2 = s ? fcv[2] : fcv[5];
        }
#pragma unroll
        for (int q1 = 0; q1 < N; ++q1) {
            const T vo = voq[q1], t1o = t1q[q1], t2o = t2q[q1], dno = dnq[q1];
            T g0, g1, g2, pen;
            if (fcmp) {
                const T bo = gow[0][q1];
                g0 = bo * w0;
                g1 = bo * w1;
                g2 = bo * w2;
                pen = fcv[6] * (bo + gnb[0][q1]);
            } else {
                g0 = gow[0][q1];
                g1 = gow[1][q1];
                g2 = gow[2][q1];
                pen = pn[q1];
            }
            const T flux = g0 * dno + g1 * t1o + g2 * t2o + fnb[q1];
            const T jump = s ? (vo - vnb[q1]) : (vnb[q1] - vo);
            const T sg = s ? T(1) : T(-1);
            const T cv = sg * (T(-0.5) * flux + pen * jump);
            const T hj = T(-0.5) * jump;
            cvq[q1] = cv;
            cnq[q1] = hj * g0;
            ct1q[q1] = hj * g1;
            ct2q[q1] = hj * g2;
        }
        contract_t2<T, N>(cvq, ct1q, A0);
        contract<T, N, 0, true>(EvenOdd<T, N>(ct2q), A1);
        contract<T, N, 0, true>(EvenOdd<T, N>(cnq), A2);
#pragma unroll
        for (int p = 0; p < N; ++p) {
            gf[rr * N + p] = A0[p];
            gf[NF + rr * N + p] = A1[p];
            gf[2 * NF + rr * N + p] = A2[p];
        }
    }
    __syncthreads();
    // step 4, lane (f, p): transposed sweep along the second direction, in
    // place: layer weights (F0) and normal-derivative weights (F1) of column p
    // in fields 0 and 1, [field][r][p]
    if (fl0) {
        if (fl) {
            T h0[N], h1[N], h2[N];
#pragma unroll
            for (int q = 0; q < N; ++q) {
                h0[q] = gf[q * N + rr];
                h1[q] = gf[NF + q * N + rr];
                h2[q] = gf[2 * NF + q * N + rr];
            }
            T f0[N], f1[N];
            contract_t2<T, N>(h0, h1, f0);
            contract<T, N, 0, true>(EvenOdd<T, N>(h2), f1);
#pragma unroll
            for (int r = 0; r < N; ++r) {
                gf[r * N + rr] = f0[r];
                gf[NF + r * N + rr] = f1[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < N; ++r) gf[r * N + rr] = gf[NF + r * N + rr] = 0;
        }
    }
    __syncthreads();
    }   // DO_FACE
    // pencil owners (j=a, l=b) add the six faces' contributions
    if (cl) {
        if constexpr (DO_FACE) {
#pragma unroll
        for (int i = 0; i < N; ++i) Y[i] = sU[cs][i + N * a + NF * b];
        const T *F = G;
        // x faces: normal coordinate i, (p, r) = (j, l)
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
            const T f0 = F[(0 + sx) * 3 * NF + b * N + a], f1 = F[(0 + sx) * 3 * NF + NF + b * N + a];
#pragma unroll
            for (int i = 0; i < N; ++i)
                Y[i] += tE<T, N>(sx, i) * f1 + ((i == (sx ? N - 1 : 0)) ? f0 : T(0));
        }
        // y faces: normal coordinate j = a, (p, r) = (i, l)
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            const T *F0 = F + (2 + sy) * 3 * NF + b * N, *F1 = F0 + NF;
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
            const T *F0 = F + (4 + sz) * 3 * NF + a * N, *F1 = F0 + NF;
            T e1 = 0;
#pragma unroll
            for (int m = 0; m < N; ++m)
                if (m == b) e1 = tE<T, N>(sz, m);
            const bool on = b == (sz ? N - 1 : 0);
#pragma unroll
            for (int i = 0; i < N; ++i) Y[i] += e1 * F1[i] + (on ? F0[i] : T(0));
        }
        }   // DO_FACE
        const int64_t o = cid * ND + N * a + NF * b;
#pragma unroll
        for (int i = 0; i < N; ++i) y[o + i] = bvec ? bvec[o + i] - Y[i] : Y[i];
    }
    // x.(A x) of the wave's cells (fixed-order wave sum), for CG's p.q; the
    // lane's input pencil comes from the copy of the input cells kept in LDS
    // (registers through the kernel would spill, and a second read from
    // memory misses the L2 on large meshes)
    if constexpr (DOT) {
        double acc = 0.0;
        if (cl) {
            const T *xo = &sXd[cs][N * a + NF * b];
#pragma unroll
            for (int i = 0; i < N; ++i) acc += (double)xo[i] * (double)Y[i];
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
        if (lane == 0) dpart[bid] = acc;
    }
}

// MODE 0: every record is a general cell; 1: every record an affine cell;
// 2: both kinds, each wave's records of one kind (groups padded to whole
// waves and interleaved), the first record's mask telling which, so that
// memory-bound waves of general cells and arithmetic-bound waves of affine
// cells share every CU
template <int N, typename T, bool DOT, int PART, int MODE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MODE ? Occ<N, T>::WA : Occ<N, T>::W,
                                                                         MODE ? Occ<N, T>::WA : Occ<N, T>::W)))
k_apply(const T *__restrict__ x, T *__restrict__ y, const T *__restrict__ bvec,
        const T *__restrict__ cell, const T *__restrict__ face, const T *__restrict__ acell,
        const T *__restrict__ kk, const T *__restrict__ aface, const T *__restrict__ fcon,
        const int32_t *__restrict__ visit, int n_cells, int nwg, double *__restrict__ dpart)
{
    constexpr int ND = Cfg<N>::ND, CPW = Cfg<N>::CPW, GS = Cfg<N>::GS;
    __shared__ T sU[CPW][ND];
    __shared__ T sG[CPW][GS];
    __shared__ T sXd[DOT ? CPW : 1][DOT ? ND : 1];   // the input cells (CG variant)
    // contiguous ranges of the traversal per XCD (workgroups are dealt
    // round-robin to the XCDs)
    const int bid = blockIdx.x;
    const int q8 = nwg / NXCD, r8 = nwg % NXCD, xcd = bid % NXCD;
    const int wg = xcd * q8 + (xcd < r8 ? xcd : r8) + bid / NXCD;
    if constexpr (MODE == 2) {
        const bool waff = visit[(int64_t)wg * CPW * 8 + 7] & 1;
        if (waff)
            apply_body<N, T, DOT, PART, true>(x, y, bvec, cell, face, acell, kk, aface, fcon, visit,
                                              n_cells, wg, bid, dpart, sU, sG, sXd);
        else
            apply_body<N, T, DOT, PART, false>(x, y, bvec, cell, face, acell, kk, aface, fcon, visit,
                                               n_cells, wg, bid, dpart, sU, sG, sXd);
    } else {
        apply_body<N, T, DOT, PART, MODE == 1>(x, y, bvec, cell, face, acell, kk, aface, fcon, visit,
                                               n_cells, wg, bid, dpart, sU, sG, sXd);
    }
}

template <int N, typename T>
hipError_t apply_n(hx_ctx *c, const T *x, T *y, const T *b, double *dpart, int *nwg_out, int part)
{
    const int cpw = Cfg<N>::CPW;
    constexpr bool F64 = std::is_same<T, double>::value;
    const T *cell = F64 ? (const T *)c->cell64 : (const T *)c->cell32;
    const T *face = F64 ? (const T *)c->face64 : (const T *)c->face32;
    const T *acell = F64 ? (const T *)c->acell64 : (const T *)c->acell32;
    const T *kk = F64 ? (const T *)c->kk64 : (const T *)c->kk32;
    const T *aface = F64 ? (const T *)c->aface64 : (const T *)c->aface32;
    const T *fcon = F64 ? (const T *)c->fc64 : (const T *)c->fc32;
    const int64_t nrec = c->n_vis_op;
    const int nwg = (int)((nrec + cpw - 1) / cpw);
    if (nwg_out) *nwg_out = nwg;
#define HX_APPLY(DOT, PART, MODE)                                                                \
    hipLaunchKernelGGL((k_apply<N, T, DOT, PART, MODE>), dim3(nwg), dim3(64), 0, c->stream, x, y, b, \
                       cell, face, acell, kk, aface, fcon, c->visit, (int)nrec, nwg, dpart)
#define HX_APPLY_MODE(MODE)                       \
    if (dpart) HX_APPLY(true, 0, MODE);          \
    else if (part == 1) HX_APPLY(false, 1, MODE); \
    else if (part == 2) HX_APPLY(false, 2, MODE); \
    else HX_APPLY(false, 0, MODE)
    if (c->vis_mode == 2) {
        HX_APPLY_MODE(2);
    } else if (c->vis_mode == 1) {
        HX_APPLY_MODE(1);
    } else {
        HX_APPLY_MODE(0);
    }
#undef HX_APPLY_MODE
#undef HX_APPLY
    return hipGetLastError();
}

template <typename T>
hipError_t apply_conforming(hx_ctx *c, const T *x, T *y, const T *b, double *dpart, int *nwg,
                            int part)
{
    switch (c->n) {
    case 2: return apply_n<2, T>(c, x, y, b, dpart, nwg, part);
    case 3: return apply_n<3, T>(c, x, y, b, dpart, nwg, part);
    case 4: return apply_n<4, T>(c, x, y, b, dpart, nwg, part);
    case 5: return apply_n<5, T>(c, x, y, b, dpart, nwg, part);
    case 6: return apply_n<6, T>(c, x, y, b, dpart, nwg, part);
    case 7: return apply_n<7, T>(c, x, y, b, dpart, nwg, part);
    case 8: return apply_n<8, T>(c, x, y, b, dpart, nwg, part);
    default: return hipErrorInvalidValue;
    }
}

// the operator, then the terms of the non-conforming quarter faces (face
// part); with quarter faces the fused x.(A x) of the CG variant is not used
// (the callers take the dot product after the whole operator)
template <typename T>
hipError_t apply_dispatch(hx_ctx *c, const T *x, T *y, const T *b, double *dpart = nullptr,
                          int *nwg = nullptr, int part = 0)
{
    hipError_t e = apply_conforming<T>(c, x, y, b, dpart, nwg, part);
    if (e != hipSuccess || c->n_hang == 0 || part == 1) return e;
    if constexpr (sizeof(T) == 8)
        return launch_hang_apply64(c, (const double *)x, (double *)y, b != nullptr);
    else
        return launch_hang_apply32(c, (const float *)x, (float *)y, b != nullptr);
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

hipError_t launch_apply_part64(hx_ctx *c, int part, const double *x, double *y)
{
    return apply_dispatch<double>(c, x, y, nullptr, nullptr, nullptr, part);
}

hipError_t launch_apply_part32(hx_ctx *c, int part, const float *x, float *y)
{
    return apply_dispatch<float>(c, x, y, nullptr, nullptr, nullptr, part);
}

// cells per wave of the operator kernel at n = k + 1 points per direction
int op_cells_per_wave(int n)
{
    switch (n) {
    case 2: return Cfg<2>::CPW;
    case 3: return Cfg<3>::CPW;
    case 4: return Cfg<4>::CPW;
    case 5: return Cfg<5>::CPW;
    case 6: return Cfg<6>::CPW;
    case 7: return Cfg<7>::CPW;
    default: return Cfg<8>::CPW;
    }
}

// y = A x and x.y (summed in a fixed order): the per-workgroup partial sums
// in c->pqpart are left there when npq is given and there are at most
// PQ_MAX of them (*npq = their count), else dst = their sum (*npq = 0)
template <typename T>
hipError_t apply_dot(hx_ctx *c, const T *x, T *y, double *dst, int *npq)
{
    if (npq) *npq = 0;
    if (c->n_hang) {
        hipError_t e = apply_dispatch<T>(c, x, y, nullptr);
        if (e != hipSuccess) return e;
        if constexpr (sizeof(T) == 8) return blas_dot(c, c->n_dofs, x, y, dst);
        else return blas_dot32(c, c->n_dofs, x, y, dst);
    }
    int nwg = 0;
    hipError_t e = apply_dispatch<T>(c, x, y, nullptr, c->pqpart, &nwg);
    if (e != hipSuccess) return e;
    if (npq && nwg <= PQ_MAX) {
        *npq = nwg;
        return hipSuccess;
    }
    return reduce_parts(c, c->pqpart, nwg, dst);
}

hipError_t launch_apply64_dot(hx_ctx *c, const double *x, double *y, double *dst, int *npq)
{
    return apply_dot<double>(c, x, y, dst, npq);
}

hipError_t launch_apply32_dot(hx_ctx *c, const float *x, float *y, double *dst, int *npq)
{
    return apply_dot<float>(c, x, y, dst, npq);
}

}  // namespace hx
