// Geometric multigrid for the SPD Helmholtz-type systems (section 3.1: CG
// preconditioned by geometric multigrid, with Chebyshev smoothing from
// Lanczos eigenvalue estimates).
//
// Levels are uniform refinements at one polynomial degree: every cell of a
// finer level fills one octant o = ox + 2 oy + 4 oz of a parent cell of the
// next coarser level, with the same axis orientation.  Prolongation writes
// the parent polynomial in the child's basis, x_child = (E_oz (x) E_oy (x)
// E_ox) x_parent with E_o[i][j] = l_j((o + xl_i)/2); restriction is its
// transpose.  Both transfers run one workgroup per coarse cell over its
// list of children, so the restriction sums without atomics; each child is
// three 1-D sweeps through LDS.  The transfers are HBM bound (8 B per fine
// dof read, plus 8 B written for the prolongation) and far cheaper than one
// operator application.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace hx {
namespace {

constexpr int MG_T = 256;

// children per pass through LDS: two buffers of CH * nd doubles, at most 32 KB
template <int N>
constexpr int mg_chunk() { return N * N * N > 125 ? 4 : 8; }

template <int N, bool RESTRICT, typename T>
__global__ __launch_bounds__(MG_T) void k_transfer(const T *__restrict__ in,
                                                   T *__restrict__ out,
                                                   const int32_t *__restrict__ cptr,
                                                   const int32_t *__restrict__ clist,
                                                   const RefTab64 *__restrict__ tab, int64_t n_coarse)
{
    constexpr int ND = N * N * N, CH = mg_chunk<N>(), NACC = (ND + MG_T - 1) / MG_T;
    __shared__ T sE[2][N * N];
    __shared__ T sA[CH][ND];
    __shared__ T sB[CH][ND];
    __shared__ T sC[ND];
    __shared__ int sChild[CH], sOct[CH];
    const int t = threadIdx.x;
    const int64_t cc = blockIdx.x;
    if (cc >= n_coarse) return;
    for (int e = t; e < 2 * N * N; e += MG_T) sE[e / (N * N)][e % (N * N)] = (T)tab->Eh[e / (N * N)][e % (N * N)];
    if (!RESTRICT)
        for (int e = t; e < ND; e += MG_T) sC[e] = in[cc * ND + e];
    T acc[NACC];
#pragma unroll
    for (int a = 0; a < NACC; ++a) acc[a] = 0;
    const int c0 = cptr[cc], c1 = cptr[cc + 1];
    for (int base = c0; base < c1; base += CH) {
        const int nch = min(CH, c1 - base);
        __syncthreads();   // the previous pass is done with sA, sB, sChild
        if (t < nch) {
            const int v = clist[base + t];
            sChild[t] = v >> 3;
            sOct[t] = v & 7;
        }
        __syncthreads();
        if (!RESTRICT) {
            // x sweep of the parent values for each child
            for (int idx = t; idx < nch * ND; idx += MG_T) {
                const int ch = idx / ND, e = idx % ND;
                const int i = e % N, bc = e / N;
                const T *E = sE[sOct[ch] & 1] + i * N;
                T s = 0;
#pragma unroll
                for (int a = 0; a < N; ++a) s += E[a] * sC[a + N * bc];
                sA[ch][e] = s;
            }
            __syncthreads();
            for (int idx = t; idx < nch * ND; idx += MG_T) {
                const int ch = idx / ND, e = idx % ND;
                const int i = e % N, j = (e / N) % N, c = e / (N * N);
                const T *E = sE[(sOct[ch] >> 1) & 1] + j * N;
                T s = 0;
#pragma unroll
                for (int b = 0; b < N; ++b) s += E[b] * sA[ch][i + N * (b + N * c)];
                sB[ch][e] = s;
            }
            __syncthreads();
            for (int idx = t; idx < nch * ND; idx += MG_T) {
                const int ch = idx / ND, e = idx % ND;
                const int ij = e % (N * N), l = e / (N * N);
                const T *E = sE[(sOct[ch] >> 2) & 1] + l * N;
                T s = 0;
#pragma unroll
                for (int c = 0; c < N; ++c) s += E[c] * sB[ch][ij + N * N * c];
                out[(int64_t)sChild[ch] * ND + e] += s;
            }
        } else {
            for (int idx = t; idx < nch * ND; idx += MG_T) {
                const int ch = idx / ND, e = idx % ND;
                sA[ch][e] = in[(int64_t)sChild[ch] * ND + e];
            }
            __syncthreads();
            // transposed x sweep: (a, j, l) <- sum_i E[i][a] r(i, j, l)
            for (int idx = t; idx < nch * ND; idx += MG_T) {
                const int ch = idx / ND, e = idx % ND;
                const int a = e % N, jl = e / N;
                const T *E = sE[sOct[ch] & 1] + a;
                T s = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) s += E[i * N] * sA[ch][i + N * jl];
                sB[ch][e] = s;
            }
            __syncthreads();
            for (int idx = t; idx < nch * ND; idx += MG_T) {
                const int ch = idx / ND, e = idx % ND;
                const int a = e % N, b = (e / N) % N, l = e / (N * N);
                const T *E = sE[(sOct[ch] >> 1) & 1] + b;
                T s = 0;
#pragma unroll
                for (int j = 0; j < N; ++j) s += E[j * N] * sB[ch][a + N * (j + N * l)];
                sA[ch][e] = s;
            }
            __syncthreads();
            // z sweep, summed over the children into the thread's outputs
#pragma unroll
            for (int q = 0; q < NACC; ++q) {
                const int e = t + q * MG_T;
                if (e < ND) {
                    const int ab = e % (N * N), c = e / (N * N);
                    for (int ch = 0; ch < nch; ++ch) {
                        const T *E = sE[(sOct[ch] >> 2) & 1] + c;
                        T s = 0;
#pragma unroll
                        for (int l = 0; l < N; ++l) s += E[l * N] * sA[ch][ab + N * N * l];
                        acc[q] += s;
                    }
                }
            }
        }
    }
    if (RESTRICT) {
#pragma unroll
        for (int q = 0; q < NACC; ++q) {
            const int e = t + q * MG_T;
            if (e < ND) out[cc * ND + e] = acc[q];
        }
    }
}

// The same transfers when every coarse cell has all eight children (the
// uniform hierarchy): child8[8 j + o] is the child in octant o of coarse cell
// j.  The tensor-product sweeps are ordered so that the children of one pair
// of octants are combined as early as possible: the restriction sweeps x on
// all eight children and adds the two x-neighbours (four results), then y
// (two), then z (one); the prolongation expands z (two), y (four), then x
// (eight).  Every thread reads its child indices itself, so the loads start
// without a barrier.  The restriction's first sweep takes one pencil pair
// per thread straight from memory, two coarse cells per workgroup while
// they fit; the prolongation runs one coarse cell per workgroup.

// coarse cells per workgroup of the dense restriction: two while one item
// per thread covers both cells' x sweep
template <int N>
constexpr int rcpb() { return 8 * N * N <= MG_T ? 2 : 1; }

template <int N, typename T>
__global__ __launch_bounds__(MG_T) __attribute__((amdgpu_waves_per_eu(N <= 5 ? 8 : 4, 8)))
void k_restrict8(const T *__restrict__ in, T *__restrict__ out,
                                                    const int32_t *__restrict__ child8,
                                                    const RefTab64 *__restrict__ tab, int64_t n_coarse)
{
    constexpr int ND = N * N * N, NF = N * N, CPB = rcpb<N>();
    __shared__ T sE[2][NF];
    __shared__ T sB[CPB][4][ND];
    __shared__ T sA[CPB][2][ND];
    const int t = threadIdx.x;
    const int64_t c0 = (int64_t)blockIdx.x * CPB;
    // the table entries requested together with the child indices
    constexpr int EPT = (2 * NF + MG_T - 1) / MG_T;
    T te[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = t + u * MG_T;
        te[u] = (T)tab->Eh[e < 2 * NF ? e / NF : 0][e < 2 * NF ? e % NF : 0];
    }
    // x: item (cell lc, pair p = oy + 2 oz, pencil jl), one per thread; the
    // two children's pencils are requested before the barrier
    const int lc = t / (4 * NF), r = t - lc * 4 * NF, p = r / NF, jl = r - p * NF;
    const bool act = lc < CPB && c0 + lc < n_coarse;
    T v0[N], v1[N];
    if (act) {
        const int64_t cc = c0 + lc;
        const T *x0 = in + (int64_t)child8[cc * 8 + 2 * p] * ND + N * jl;
        const T *x1 = in + (int64_t)child8[cc * 8 + 2 * p + 1] * ND + N * jl;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            v0[i] = x0[i];
            v1[i] = x1[i];
        }
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = t + u * MG_T;
        if (e < 2 * NF) sE[e / NF][e % NF] = te[u];
    }
    __syncthreads();
    if (act) {
#pragma unroll 1
        for (int a = 0; a < N; ++a) {
            T s = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) s += sE[0][i * N + a] * v0[i] + sE[1][i * N + a] * v1[i];
            sB[lc][p][a + N * jl] = s;
        }
    }
    __syncthreads();
    // y: (a, b, l) of oz, summed over oy
#pragma unroll 1
    for (int it = t; it < CPB * 2 * ND; it += MG_T) {
        const int lc2 = it / (2 * ND), r2 = it - lc2 * 2 * ND, q = r2 / ND, e = r2 - q * ND;
        if (c0 + lc2 >= n_coarse) continue;
        const int a = e % N, b = (e / N) % N, l = e / NF;
        T s = 0;
#pragma unroll
        for (int j = 0; j < N; ++j)
            s += sE[0][j * N + b] * sB[lc2][2 * q][a + N * (j + N * l)] +
                 sE[1][j * N + b] * sB[lc2][2 * q + 1][a + N * (j + N * l)];
        sA[lc2][q][e] = s;
    }
    __syncthreads();
    // z: summed over oz
#pragma unroll 1
    for (int it = t; it < CPB * ND; it += MG_T) {
        const int lc2 = it / ND, e = it - lc2 * ND;
        const int64_t cc = c0 + lc2;
        if (cc >= n_coarse) continue;
        const int ab = e % NF, c = e / NF;
        T s = 0;
#pragma unroll
        for (int l = 0; l < N; ++l)
            s += sE[0][l * N + c] * sA[lc2][0][ab + NF * l] + sE[1][l * N + c] * sA[lc2][1][ab + NF * l];
        out[cc * ND + e] = s;
    }
}

template <int N, typename T>
__global__ __launch_bounds__(MG_T) void k_prolong8(const T *__restrict__ in, T *__restrict__ out,
                                                   const int32_t *__restrict__ child8,
                                                   const RefTab64 *__restrict__ tab, int64_t n_coarse)
{
    constexpr int ND = N * N * N, NF = N * N;
    __shared__ T sE[2][NF];
    __shared__ T sC[ND];
    __shared__ T sZ[2][ND];
    __shared__ T sY[4][ND];
    const int t = threadIdx.x;
    const int64_t cc = blockIdx.x;
    if (cc >= n_coarse) return;
    // every load up front: the table, the coarse values, the eight child
    // indices, then the fine values this thread adds to (their latency
    // overlaps the z and y sweeps)
    constexpr int EPT = (2 * NF + MG_T - 1) / MG_T, CPT = (ND + MG_T - 1) / MG_T,
                  OPT = (8 * ND + MG_T - 1) / MG_T;
    T te[EPT], tc[CPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = t + u * MG_T;
        te[u] = (T)tab->Eh[e < 2 * NF ? e / NF : 0][e < 2 * NF ? e % NF : 0];
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int e = t + u * MG_T;
        tc[u] = in[cc * ND + (e < ND ? e : 0)];
    }
    const int4 *c4 = reinterpret_cast<const int4 *>(child8 + cc * 8);
    const int4 k0 = c4[0], k1 = c4[1];
    const int32_t kids[8] = {k0.x, k0.y, k0.z, k0.w, k1.x, k1.y, k1.z, k1.w};
    T fo[OPT];
#pragma unroll
    for (int u = 0; u < OPT; ++u) {
        const int idx = t + u * MG_T;
        const int o = idx < 8 * ND ? idx / ND : 0, e = idx < 8 * ND ? idx - o * ND : 0;
        fo[u] = out[(int64_t)kids[o] * ND + e];
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
        const int e = t + u * MG_T;
        if (e < 2 * NF) sE[e / NF][e % NF] = te[u];
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int e = t + u * MG_T;
        if (e < ND) sC[e] = tc[u];
    }
    __syncthreads();
    // z: (a, b, l) for oz = 0, 1
    for (int idx = t; idx < 2 * ND; idx += MG_T) {
        const int q = idx / ND, e = idx - q * ND;
        const int ab = e % NF, l = e / NF;
        T s = 0;
#pragma unroll
        for (int c = 0; c < N; ++c) s += sE[q][l * N + c] * sC[ab + NF * c];
        sZ[q][e] = s;
    }
    __syncthreads();
    // y: (a, j, l) for p = oy + 2 oz
    for (int idx = t; idx < 4 * ND; idx += MG_T) {
        const int p = idx / ND, e = idx - p * ND;
        const int a = e % N, j = (e / N) % N, l = e / NF;
        const T *E = sE[p & 1] + j * N;
        const T *src = sZ[p >> 1];
        T s = 0;
#pragma unroll
        for (int b = 0; b < N; ++b) s += E[b] * src[a + N * (b + N * l)];
        sY[p][e] = s;
    }
    __syncthreads();
    // x: (i, j, l) of octant o = ox + 2 p, added to the child
#pragma unroll
    for (int u = 0; u < OPT; ++u) {
        const int idx = t + u * MG_T;
        if (idx >= 8 * ND) break;
        const int o = idx / ND, e = idx - o * ND;
        const int i = e % N, jl = e / N;
        const T *E = sE[o & 1] + i * N;
        const T *src = sY[o >> 1];
        T s = 0;
#pragma unroll
        for (int a = 0; a < N; ++a) s += E[a] * src[a + N * jl];
        out[(int64_t)kids[o] * ND + e] = fo[u] + s;
    }
}

template <bool RESTRICT, typename T>
hipError_t transfer(hx_ctx *c, const T *in, T *out)
{
    const int64_t nc = c->mg_nc;
    if (nc == 0) return hipSuccess;
    const dim3 g((unsigned)nc), b(MG_T);
#define HX_MG_CASE(NN)                                                                           \
    case NN:                                                                                     \
        if (c->mg_child8 && RESTRICT)                                                            \
            hipLaunchKernelGGL((k_restrict8<NN, T>), dim3((unsigned)((nc + rcpb<NN>() - 1) /      \
                                                                   rcpb<NN>())),                 \
                               b, 0, c->stream, in, out, c->mg_child8, c->ref, nc);              \
        else if (c->mg_child8)                                                                   \
            hipLaunchKernelGGL((k_prolong8<NN, T>), g, b, 0, c->stream, in, out, c->mg_child8,   \
                               c->ref, nc);                                                      \
        else                                                                                     \
            hipLaunchKernelGGL((k_transfer<NN, RESTRICT, T>), g, b, 0, c->stream, in, out,       \
                               c->mg_cptr, c->mg_clist, c->ref, nc);                             \
        break;
    switch (c->n) {
        HX_MG_CASE(2) HX_MG_CASE(3) HX_MG_CASE(4) HX_MG_CASE(5) HX_MG_CASE(6) HX_MG_CASE(7)
        HX_MG_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef HX_MG_CASE
    return hipGetLastError();
}

}  // namespace

hipError_t mg_restrict64(hx_ctx *c, const double *r_fine, double *b_coarse)
{
    return transfer<true, double>(c, r_fine, b_coarse);
}

hipError_t mg_prolong_add64(hx_ctx *c, const double *x_coarse, double *x_fine)
{
    return transfer<false, double>(c, x_coarse, x_fine);
}

// x = V b: Chebyshev smoothing from zero, the restricted residual solved by
// the V-cycle of the next coarser level and its prolongation added, then the
// same Chebyshev iteration continued from the corrected x (which applies the
// same polynomial to the updated residual and keeps V symmetric); the
// coarsest level applies its own Chebyshev polynomial.  All levels share one
// stream, so no synchronisation is needed between them.
hipError_t mg_vcycle64(hx_ctx *c, const double *b, double *x)
{
    if (!c->mg_coarse) return cheb_iterate64(c, b, x, true);
    hx_ctx *C = c->mg_coarse;
    const int64_t n = c->n_dofs;
    double *r = c->mgw + 2 * n;
    double *bc = C->mgw, *xc = C->mgw + C->n_dofs;
    hipError_t e = cheb_iterate64(c, b, x, true);
    if (e == hipSuccess) e = launch_apply64(c, x, r, b);      // r = b - A x
    if (e == hipSuccess) e = transfer<true, double>(c, r, bc);
    if (e == hipSuccess) e = mg_vcycle64(C, bc, xc);
    if (e == hipSuccess) e = transfer<false, double>(c, xc, x);
    if (e == hipSuccess) e = cheb_iterate64(c, b, x, false);
    return e;
}

namespace {
hipError_t vcycle32(hx_ctx *c, const float *b, float *x)
{
    if (!c->mg_coarse) return cheb_iterate32(c, b, x, true);
    hx_ctx *C = c->mg_coarse;
    const int64_t n = c->n_dofs;
    float *r = c->mgw32 + 2 * n;
    float *bc = C->mgw32, *xc = C->mgw32 + C->n_dofs;
    hipError_t e = cheb_iterate32(c, b, x, true);
    if (e == hipSuccess) e = launch_apply32(c, x, r, b);
    if (e == hipSuccess) e = transfer<true, float>(c, r, bc);
    if (e == hipSuccess) e = vcycle32(C, bc, xc);
    if (e == hipSuccess) e = transfer<false, float>(c, xc, x);
    if (e == hipSuccess) e = cheb_iterate32(c, b, x, false);
    return e;
}
}  // namespace

// The FP32 V-cycle as the preconditioner of an FP64 Krylov method: the FP64
// residual is rounded to FP32, the cycle runs on the FP32 operator data, and
// its result is widened again.  The rounding makes the preconditioner
// slightly non-linear (relative perturbations of order 1e-7); CG tolerates
// that in practice and FGMRES by construction.
hipError_t mg_vcycle_mixed(hx_ctx *c, const double *r, double *z)
{
    const int64_t n = c->n_dofs;
    float *b32 = c->mgw32, *x32 = c->mgw32 + n;
    hipError_t e = blas_cast64to32(c, n, r, b32, nullptr);
    if (e == hipSuccess) e = vcycle32(c, b32, x32);
    if (e == hipSuccess) e = blas_cast32to64(c, n, x32, z, nullptr);
    return e;
}

// the FP32 cycle on the finest level's own vectors: input in mgw32[0, n),
// output in mgw32[n, 2n) (the fused CG step writes the input itself)
hipError_t mg_vcycle32_resident(hx_ctx *c)
{
    const int64_t n = c->n_dofs;
    return vcycle32(c, c->mgw32, c->mgw32 + n);
}

}  // namespace hx
