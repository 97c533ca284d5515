// Krylov building blocks on one stream: deterministic two-stage reductions
// (wave64 shuffles, then a fixed-order LDS tree; the stage-1 partition
// depends only on n, so results are bitwise reproducible), block dot products
// and block updates for classical Gram-Schmidt, fused CG updates that read
// their scalars from device memory (no host round trip), casts.
#include "common.hpp"
#include "sum256.hpp"

namespace hx {
namespace {

constexpr int RT = 256;          // threads of a reduction block
constexpr int RED_MAX = 1024;    // max stage-1 blocks
constexpr int MC = 8;            // vectors per block-dot pass

// eight elements per thread, or two on small systems (whose few blocks
// would otherwise be latency bound); at most RED_MAX
inline int red_blocks(int64_t n)
{
    int64_t b = (n + RT * 8 - 1) / (RT * 8);
    if (b < 256) b = (n + RT * 2 - 1) / (RT * 2);
    if (b < 1) b = 1;
    if (b > RED_MAX) b = RED_MAX;
    return (int)b;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// sum over the block in a fixed order; result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double *sh)
{
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    __syncthreads();
    return s;
}

template <typename T>
__global__ void __launch_bounds__(RT) k_dot1(int64_t n, const T *__restrict__ x,
                                             const T *__restrict__ y, double *part)
{
    __shared__ double sh[RT / 64];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RT;
    for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += stride)
        s += (double)x[i] * (double)y[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// stage 2: block v sums part[v*ld + 0..nb)
__global__ void __launch_bounds__(RT) k_red2(const double *__restrict__ part, int nb, int ld,
                                             double *dst)
{
    __shared__ double sh[RT / 64];
    double s = 0.0;
    const double *p = part + (int64_t)blockIdx.x * ld;
    for (int i = threadIdx.x; i < nb; i += RT) s += p[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) dst[blockIdx.x] = s;
}

// block dot: part[(v0+k)*ld + blk] = sum_i V[v0+k][i] w[i], k < mc
__global__ void __launch_bounds__(RT) k_mdot1(int64_t n, int v0, int mc,
                                              const double *__restrict__ V, int64_t ldv,
                                              const double *__restrict__ w, double *part, int ld)
{
    __shared__ double sh[RT / 64];
    double s[MC];
#pragma unroll
    for (int k = 0; k < MC; ++k) s[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RT;
    for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += stride) {
        const double wi = w[i];
#pragma unroll
        for (int k = 0; k < MC; ++k)
            if (k < mc) s[k] += V[(int64_t)(v0 + k) * ldv + i] * wi;
    }
#pragma unroll
    for (int k = 0; k < MC; ++k) {
        if (k >= mc) break;
        const double r = block_sum(s[k], sh);
        if (threadIdx.x == 0) part[(int64_t)(v0 + k) * ld + blockIdx.x] = r;
    }
}

// ---------------------------------------------------------------------------
// One step of classical Gram-Schmidt with the second pass delayed by one step
// (see solver.cpp), in four launches.  V[j] holds the tentative vector t of
// the previous step, w = A z_j.
//
// k_dcgs_dot: per workgroup, partial block dots of [V_0 .. V_{j-1}, t] with t
// and with w.  k_dcgs_coef sums them in a fixed order and derives the step's
// scalars: sc[0..j): c = V_{j-1}^T t, sc[j]: t.t, sc[64..64+j): h = V_{j-1}^T w,
// sc[64+j]: t.w, sc[DC_CW + k] = h_k - c_k hj/rho, sc[DC_S + 0..4] = 1/rho,
// hj/rho, rho, hj, flag (1 if t lies in the span of V_{j-1} to working
// precision).
// ---------------------------------------------------------------------------
constexpr int DC_CW = 300, DC_S = 364;
constexpr int DMC = 32;           // most basis vectors per pass of the block kernels
constexpr int DC_LD = 1024;       // partial-sum row stride (max workgroups per chunk)

// rows r < nrows of part (stride ld, nb <= 1024 columns) summed in a fixed
// order, one wave per row, each wave's rows two at a time with all their
// loads in flight together; result in out[r] (LDS)
__device__ void sum_rows(const double *__restrict__ part, int nrows, int nb, int ld, double *out)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int r0 = wv; r0 < nrows; r0 += 2 * nw) {
        double s[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int r = r0 + q * nw;
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int p = lane + 64 * u;
                v[u] = (r < nrows && p < nb) ? part[(int64_t)r * ld + p] : 0.0;
            }
            double a = 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u) a += v[u];
            s[q] = a;
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const double t = wave_sum(s[q]);
            const int r = r0 + q * nw;
            if (lane == 0 && r < nrows) out[r] = t;
        }
    }
}

// MC: vectors per workgroup row (a multiple of 4 at least the chunk's
// count, so few loads are wasted on padding); NT: streaming loads of the
// basis (vectors far larger than the caches; on small systems the basis is
// read again from the caches at the next step)
template <int MC, bool NT>
__global__ void __launch_bounds__(RT) k_dcgs_dot(int64_t n, int j, const double *__restrict__ V,
                                                 int64_t ldv, const double *__restrict__ w,
                                                 double *part)
{
    __shared__ double wsum[RT / 64][2 * MC];
    const int m = j + 1;
    const int v0 = blockIdx.y * MC;
    const int mc = (m - v0) < MC ? (m - v0) : MC;
    const double *t = V + (int64_t)j * ldv;
    double sa[MC], sb[MC];
#pragma unroll
    for (int k = 0; k < MC; ++k) sa[k] = sb[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RT;
    // rows past the chunk's last vector repeat that vector (same cache
    // lines, results unused), so the loads issue without branches
    const double *rows[MC];
#pragma unroll
    for (int k = 0; k < MC; ++k) rows[k] = V + (int64_t)(v0 + (k < mc ? k : mc - 1)) * ldv;
    for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += stride) {
        const double ai = t[i], bi = w[i];
        double v[MC];
#pragma unroll
        for (int k = 0; k < MC; ++k) v[k] = NT ? __builtin_nontemporal_load(rows[k] + i) : rows[k][i];
        // every load in flight before the arithmetic (the scheduler would
        // interleave them with the multiply-adds to save registers)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < MC; ++k) {
            sa[k] += v[k] * ai;
            sb[k] += v[k] * bi;
        }
    }
    // per-wave sums, then the waves in a fixed order
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < MC; ++k) {
        const double ra = wave_sum(sa[k]), rb = wave_sum(sb[k]);
        if (lane == 0) {
            wsum[wv][k] = ra;
            wsum[wv][MC + k] = rb;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < 2 * mc) {
        const int k = threadIdx.x < mc ? threadIdx.x : threadIdx.x - mc;
        const int col = threadIdx.x < mc ? k : MC + k;
        double r = 0.0;
        for (int q = 0; q < RT / 64; ++q) r += wsum[q][col];
        const int row = threadIdx.x < mc ? v0 + k : m + v0 + k;
        part[(int64_t)row * DC_LD + blockIdx.x] = r;
    }
}

// k_dcgs_coef (one workgroup of 1024): the 2(j+1) dot products from the
// nb partial sums of each, in a fixed order, and the step's scalars
__global__ void __launch_bounds__(1024) k_dcgs_coef(int j, int nb, const double *__restrict__ part,
                                                    double *sc, double *hout)
{
    __shared__ double sums[2 * 64];
    const int m = j + 1;
    sum_rows(part, 2 * m, nb, DC_LD, sums);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double *ca = sums, *cb = sums + m;
    double cc = 0.0, ch = 0.0;
    for (int k = 0; k < j; ++k) {
        cc += ca[k] * ca[k];
        ch += ca[k] * cb[k];
    }
    const double r2 = ca[j] - cc;
    double flag = 0.0, rho;
    if (r2 > 0.0 && r2 >= 1e-12 * ca[j]) {
        rho = sqrt(r2);
    } else {
        flag = 1.0;
        rho = ca[j] > 0.0 ? sqrt(ca[j]) : 1.0;
    }
    const double hj = (cb[j] - ch) / rho;
    for (int k = 0; k <= j; ++k) {
        sc[k] = ca[k];
        sc[64 + k] = cb[k];
    }
    for (int k = 0; k < j; ++k) sc[DC_CW + k] = cb[k] - ca[k] * (hj / rho);
    sc[DC_S + 0] = 1.0 / rho;
    sc[DC_S + 1] = hj / rho;
    sc[DC_S + 2] = rho;
    sc[DC_S + 3] = hj;
    sc[DC_S + 4] = flag;
    if (hout) {
        for (int k = 0; k <= j; ++k) {
            hout[k] = ca[k];
            hout[64 + k] = cb[k];
        }
        for (int k = 0; k < 5; ++k) hout[DC_S + k] = sc[DC_S + k];
    }
}

// k_dcgs_update: with t = V[j],
//   V[j] <- (t - V_{j-1} c) / rho,  w <- w - V_{j-1} cw - t hj/rho
// (reads V_{j-1} once, MC vectors at a time with all their loads in flight;
// rows past V_{j-1} repeat its last vector with coefficient 0), and per
// workgroup the partial sum of the new |w|^2.  Vr: V_0 .. V_{j-1} (read
// only), t: V_j; the two do not overlap.
template <int MC>
__global__ void __launch_bounds__(RT) k_dcgs_update(int64_t n, int j, const double *__restrict__ Vr,
                                                    int64_t ldv, double *__restrict__ t,
                                                    const double *__restrict__ sc,
                                                    double *__restrict__ w, double *part,
                                                    double *hpart)
{
    __shared__ double sh[RT / 64];
    __shared__ double cs[64], cws[64];
    const int jp = (j + MC - 1) / MC * MC;
    for (int k = threadIdx.x; k < jp; k += RT) {
        cs[k] = k < j ? sc[k] : 0.0;
        cws[k] = k < j ? sc[DC_CW + k] : 0.0;
    }
    __syncthreads();
    const double irho = sc[DC_S + 0], hr = sc[DC_S + 1];
    double nu = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RT;
    for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += stride) {
        const double ti = t[i], wi = w[i];
        double sv = 0.0, sw = 0.0;
        for (int k0 = 0; k0 < j; k0 += MC) {
            double v[MC];
#pragma unroll
            for (int k = 0; k < MC; ++k) {
                const int r = k0 + k < j ? k0 + k : j - 1;
                v[k] = Vr[(int64_t)r * ldv + i];
            }
            __builtin_amdgcn_sched_barrier(0);   // every load in flight first
#pragma unroll
            for (int k = 0; k < MC; ++k) {
                sv += v[k] * cs[k0 + k];
                sw += v[k] * cws[k0 + k];
            }
        }
        t[i] = (ti - sv) * irho;
        const double wn = wi - sw - ti * hr;
        w[i] = wn;
        nu += wn * wn;
    }
    nu = block_sum(nu, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = nu;
        if (hpart) hpart[blockIdx.x] = nu;
    }
}

// k_dcgs_scale: every workgroup sums the nb partial sums of |w|^2 (sum256)
// and writes its slice of V[j+1] = w / |w|; workgroup 0 also stores |w|^2 in
// *dst
__global__ void __launch_bounds__(RT) k_dcgs_scale(int64_t n, int nb, const double *__restrict__ part,
                                                   const double *__restrict__ w, double *v, double *dst)
{
    __shared__ double sh[4];
    const double s2 = sum256(part, nb, sh);
    if (blockIdx.x == 0 && threadIdx.x == 0) dst[0] = s2;
    const double inv = 1.0 / sqrt(s2);
    const int64_t stride = (int64_t)gridDim.x * RT;
    for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += stride) v[i] = w[i] * inv;
}

// w += sign * sum_k h[k] V[k]
__global__ void k_mupdate(int64_t n, int m, const double *__restrict__ V, int64_t ldv,
                          const double *__restrict__ h, double sign, double *w)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += h[k] * V[(int64_t)k * ldv + i];
    w[i] += sign * s;
}

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// mode 0: y = s x, 1: y = x / s, 2: y = x / sqrt(s)
__global__ void k_scale_copy(int64_t n, const double *__restrict__ s, int mode,
                             const double *__restrict__ x, double *y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = s[0];
    y[i] = mode == 0 ? v * x[i] : (mode == 1 ? x[i] / v : x[i] / sqrt(v));
}

// y = (float)(x * scale), scale = 1/sqrt(s) if s != null
__global__ void k_cast64to32(int64_t n, const double *__restrict__ x, float *y,
                             const double *__restrict__ s)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double f = s ? 1.0 / sqrt(s[0]) : 1.0;
    y[i] = (float)(x[i] * f);
}

// y = (double)x * scale, scale = sqrt(s) if s != null
__global__ void k_cast32to64(int64_t n, const float *__restrict__ x, double *y,
                             const double *__restrict__ s)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double f = s ? sqrt(s[0]) : 1.0;
    y[i] = (double)x[i] * f;
}

template <typename T>
__global__ void k_fill(int64_t n, T v, T *y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

__global__ void k_copy(int64_t n, const double *__restrict__ x, double *y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i];
}

// ---- FP32 CG with device scalars: sc[0] = rz (current), sc[1] = p.q,
// sc[2] = new rz.  x += a p, r -= a q with a = sc[0]/p.q; p.q is the
// fixed-order sum of pqp[0..npq) when pqp is given, else sc[1].
// 256 threads per block.
__global__ void __launch_bounds__(256) k_cg_x(int64_t n, float *x, float *r,
                                              const float *__restrict__ p,
                                              const float *__restrict__ q,
                                              const double *__restrict__ sc,
                                              const double *__restrict__ pqp, int npq)
{
    __shared__ double shq[4];
    const double pq = pqp ? sum256(pqp, npq, shq) : sc[1];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float a = (float)(pq != 0.0 ? sc[0] / pq : 0.0);
    x[i] += a * p[i];
    r[i] -= a * q[i];
}

// p = z + (sc[2]/sc[0]) p
__global__ void k_cg_p(int64_t n, const float *__restrict__ z, float *p,
                       const double *__restrict__ sc)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float bt = (float)(sc[0] != 0.0 ? sc[2] / sc[0] : 0.0);
    p[i] = z[i] + bt * p[i];
}

__global__ void k_shift(double *sc)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) sc[0] = sc[2];
}

// ---- fused CG steps, FP64 or FP32 vectors, scalars on the device:
// sc[0] = r.z (current), sc[1] = p.q, sc[2] = new r.z, sc[3] = new r.r.
// x += a p, r -= a q with a = sc[0] / p.q (0 when p.q is exactly 0: the
// step in flight after exact convergence), z = dinv r (or z = r), and the
// per-block partial sums of r.z and r.r in part[blk], part[ld + blk].
// p.q is the fixed-order sum of pqp[0..npq) when pqp is given, else sc[1].
template <typename T>
__global__ void __launch_bounds__(RT) k_cg_elem(int64_t n, T *x, T *r, const T *__restrict__ p,
                                                const T *__restrict__ q, T *z,
                                                const T *__restrict__ dinv,
                                                const double *__restrict__ sc, double *part, int ld,
                                                float *r32, const double *__restrict__ pqp, int npq)
{
    static_assert(RT == 256, "sum256 needs 256 threads");
    __shared__ double sh[RT / 64];
    __shared__ double shq[4];
    const double pq = pqp ? sum256(pqp, npq, shq) : sc[1];
    const T al = (T)(pq != 0.0 ? sc[0] / pq : 0.0);
    double rz = 0.0, rr = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RT;
    for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += stride) {
        const T rv = r[i] - al * q[i];
        x[i] += al * p[i];
        r[i] = rv;
        const T zv = dinv ? dinv[i] * rv : rv;
        if (r32) r32[i] = (float)rv;   // the FP32 V-cycle's input in place of z
        else z[i] = zv;
        rz += (double)rv * (double)zv;
        rr += (double)rv * (double)rv;
    }
    rz = block_sum(rz, sh);
    rr = block_sum(rr, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = rz;
        part[ld + blockIdx.x] = rr;
    }
}

// z = (double) x32 and per-block partial sums of r.z (the FP32 V-cycle's
// output widened and dotted in one pass)
__global__ void __launch_bounds__(RT) k_widen_dot(int64_t n, const float *__restrict__ x32,
                                                  const double *__restrict__ r, double *z,
                                                  double *part)
{
    __shared__ double sh[RT / 64];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RT;
    for (int64_t i = blockIdx.x * (int64_t)RT + threadIdx.x; i < n; i += stride) {
        const double zv = (double)x32[i];
        z[i] = zv;
        s += r[i] * zv;
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = z + (sc[2] / sc[0]) p
template <typename T>
__global__ void k_cg_pt(int64_t n, const T *__restrict__ z, T *p, const double *__restrict__ sc,
                        int beta_ready)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T bt = (T)(beta_ready ? sc[5] : (sc[0] != 0.0 ? sc[2] / sc[0] : 0.0));
    p[i] = z[i] + bt * p[i];
}

// p = z + beta p with beta = new r.z / sc[cur]: every workgroup sums the
// fused step's nb partial sums of r.z (row 0 of part) in the same fixed
// order; workgroup 0 also sums r.r (row 1) and writes the new r.z to
// sc[2 - cur] (the slot no workgroup reads here), r.r to sc[3] and, when
// host is given (device view of pinned memory), to *host.  256 threads.
template <typename T>
__global__ void __launch_bounds__(256) k_cg_pt_red(int64_t n, const T *__restrict__ z, T *p,
                                                   const double *__restrict__ part, int nb, int ld,
                                                   double *sc, int cur, double *host)
{
    __shared__ double sh[4];
    const double rz = sum256(part, nb, sh);
    const double old = sc[cur];
    const T bt = (T)(old != 0.0 ? rz / old : 0.0);
    if (blockIdx.x == 0) {
        const double rr = sum256(part + ld, nb, sh);
        if (threadIdx.x == 0) {
            sc[2 - cur] = rz;
            sc[3] = rr;
            if (host) *host = rr;
        }
    }
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + bt * p[i];
}

// stage 2 of a fused CG step whose z is final: workgroup 0 sums r.z (row 0
// of part), workgroup 1 r.r (row 1); then beta = new r.z / old r.z goes to
// sc[5] and the new r.z to sc[2] and sc[0] (so no separate shift is needed),
// r.r to sc[3] and, when host is given (device view of pinned memory), to
// *host.  The sums take k_red2's order.
__global__ void __launch_bounds__(RT) k_red_cg(const double *__restrict__ part, int nb, int ld,
                                               double *sc, double *host)
{
    __shared__ double sh[RT / 64];
    double s = 0.0;
    const double *p = part + (int64_t)blockIdx.x * ld;
    for (int i = threadIdx.x; i < nb; i += RT) s += p[i];
    s = block_sum(s, sh);
    if (threadIdx.x != 0) return;
    if (blockIdx.x == 0) {
        const double old = sc[0];
        sc[5] = old != 0.0 ? s / old : 0.0;
        sc[2] = s;
        sc[0] = s;
    } else {
        sc[3] = s;
        if (host) *host = s;
    }
}

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t blas_dot(hx_ctx *c, int64_t n, const double *x, const double *y, double *dst)
{
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_dot1<double>, dim3(nb), dim3(RT), 0, c->stream, n, x, y, c->red);
    hipLaunchKernelGGL(k_red2, dim3(1), dim3(RT), 0, c->stream, c->red, nb, RED_MAX, dst);
    return hipGetLastError();
}

hipError_t blas_dot32(hx_ctx *c, int64_t n, const float *x, const float *y, double *dst)
{
    const int nb = red_blocks(n);
    hipLaunchKernelGGL(k_dot1<float>, dim3(nb), dim3(RT), 0, c->stream, n, x, y, c->red);
    hipLaunchKernelGGL(k_red2, dim3(1), dim3(RT), 0, c->stream, c->red, nb, RED_MAX, dst);
    return hipGetLastError();
}

hipError_t blas_mdot(hx_ctx *c, int64_t n, int m, const double *V, int64_t ldv, const double *w,
                     double *dst)
{
    const int nb = red_blocks(n);
    for (int v0 = 0; v0 < m; v0 += MC) {
        const int mc = (m - v0) < MC ? (m - v0) : MC;
        hipLaunchKernelGGL(k_mdot1, dim3(nb), dim3(RT), 0, c->stream, n, v0, mc, V, ldv, w, c->red,
                           RED_MAX);
    }
    hipLaunchKernelGGL(k_red2, dim3(m), dim3(RT), 0, c->stream, c->red, nb, RED_MAX, dst);
    return hipGetLastError();
}

// one delayed-reorthogonalisation step (see k_dcgs_dot): finalises V[j],
// projects w, stores |w|^2 in sc[128] and the tentative next vector w/|w| in
// V[j+1]; j < 64
hipError_t blas_dcgs(hx_ctx *c, int64_t n, int j, double *V, int64_t ldv, double *w, double *sc,
                     double *host_out, bool scale, int *nb_out)
{
    if (j < 0 || j >= 64) return hipErrorInvalidValue;
    // four elements per thread, or one on small systems (whose few
    // workgroups would otherwise be latency bound)
    int64_t want = (n + RT * 4 - 1) / (RT * 4);
    if (want < 256) want = (n + RT - 1) / RT;
    const int nb = (int)(want < 1 ? 1 : (want > DC_LD ? DC_LD : want));
    // the dot's vectors in as few chunks of at most DMC as possible, each
    // padded to a multiple of 4
    const int nch = (j + 1 + DMC - 1) / DMC;
    const int per = (j + 1 + nch - 1) / nch;
    int64_t want2 = (n + RT * 2 - 1) / (RT * 2);
    if (want2 < 256) want2 = (n + RT - 1) / RT;
    const int nb2 = (int)(want2 < 1 ? 1 : (want2 > RED_MAX ? RED_MAX : want2));
    double *hp = host_out ? host_out + FG_PART : nullptr;
    double *t = V + (int64_t)j * ldv;
    const bool nt = n >= ((int64_t)1 << 23);   // 64 MB vectors and up
#define HX_DCGS(MC)                                                                                \
    case MC:                                                                                       \
        if (nt)                                                                                    \
            hipLaunchKernelGGL((k_dcgs_dot<MC, true>), dim3(nb, nch), dim3(RT), 0, c->stream, n, j, \
                               V, ldv, w, c->dpart);                                               \
        else                                                                                       \
            hipLaunchKernelGGL((k_dcgs_dot<MC, false>), dim3(nb, nch), dim3(RT), 0, c->stream, n,   \
                               j, V, ldv, w, c->dpart);                                            \
        hipLaunchKernelGGL(k_dcgs_coef, dim3(1), dim3(1024), 0, c->stream, j, nb, c->dpart, sc,     \
                           host_out);                                                              \
        hipLaunchKernelGGL(k_dcgs_update<MC>, dim3(nb2), dim3(RT), 0, c->stream, n, j, V, ldv, t,   \
                           sc, w, c->red + RED_WPART, hp);                                         \
        break
    switch ((per + 3) / 4 * 4) {
        HX_DCGS(4);
        HX_DCGS(8);
        HX_DCGS(12);
        HX_DCGS(16);
        HX_DCGS(20);
        HX_DCGS(24);
        HX_DCGS(28);
        HX_DCGS(32);
    default: return hipErrorInvalidValue;
    }
#undef HX_DCGS
    if (scale) {
        const int64_t want3 = (n + RT * 4 - 1) / (RT * 4);
        const int nb3 = (int)(want3 < 1 ? 1 : (want3 > 4096 ? 4096 : want3));
        hipLaunchKernelGGL(k_dcgs_scale, dim3(nb3), dim3(RT), 0, c->stream, n, nb2, c->red + RED_WPART,
                           w, V + (int64_t)(j + 1) * ldv, sc + 128);
    }
    if (nb_out) *nb_out = nb2;
    return hipGetLastError();
}

hipError_t blas_mupdate(hx_ctx *c, int64_t n, int m, const double *V, int64_t ldv, const double *h,
                        double sign, double *w)
{
    hipLaunchKernelGGL(k_mupdate, dim3(nb256(n)), dim3(256), 0, c->stream, n, m, V, ldv, h, sign, w);
    return hipGetLastError();
}

hipError_t blas_lincomb(hx_ctx *c, int64_t n, int m, const double *Z, int64_t ldz,
                        const double *y_dev, double *x)
{
    return blas_mupdate(c, n, m, Z, ldz, y_dev, 1.0, x);
}

hipError_t blas_axpby(hx_ctx *c, int64_t n, double a, const double *x, double b, double *y)
{
    hipLaunchKernelGGL(k_axpby, dim3(nb256(n)), dim3(256), 0, c->stream, n, a, x, b, y);
    return hipGetLastError();
}

hipError_t blas_scale_copy(hx_ctx *c, int64_t n, const double *s_dev, int mode, const double *x,
                           double *y)
{
    hipLaunchKernelGGL(k_scale_copy, dim3(nb256(n)), dim3(256), 0, c->stream, n, s_dev, mode, x, y);
    return hipGetLastError();
}

hipError_t blas_cast64to32(hx_ctx *c, int64_t n, const double *x, float *y, const double *s_dev)
{
    hipLaunchKernelGGL(k_cast64to32, dim3(nb256(n)), dim3(256), 0, c->stream, n, x, y, s_dev);
    return hipGetLastError();
}

hipError_t blas_cast32to64(hx_ctx *c, int64_t n, const float *x, double *y, const double *s_dev)
{
    hipLaunchKernelGGL(k_cast32to64, dim3(nb256(n)), dim3(256), 0, c->stream, n, x, y, s_dev);
    return hipGetLastError();
}

hipError_t blas_copy(hx_ctx *c, int64_t n, const double *x, double *y)
{
    hipLaunchKernelGGL(k_copy, dim3(nb256(n)), dim3(256), 0, c->stream, n, x, y);
    return hipGetLastError();
}

hipError_t blas_fill(hx_ctx *c, int64_t n, double v, double *y)
{
    hipLaunchKernelGGL(k_fill<double>, dim3(nb256(n)), dim3(256), 0, c->stream, n, v, y);
    return hipGetLastError();
}

hipError_t blas_fill32(hx_ctx *c, int64_t n, float v, float *y)
{
    hipLaunchKernelGGL(k_fill<float>, dim3(nb256(n)), dim3(256), 0, c->stream, n, v, y);
    return hipGetLastError();
}

hipError_t cg32_step_x(hx_ctx *c, int64_t n, float *x, float *r, const float *p, const float *q,
                       double *sc, const double *pqp, int npq)
{
    hipLaunchKernelGGL(k_cg_x, dim3(nb256(n)), dim3(256), 0, c->stream, n, x, r, p, q, sc, pqp,
                       npq);
    return hipGetLastError();
}

hipError_t cg32_step_p(hx_ctx *c, int64_t n, const float *z, float *p, double *sc)
{
    hipLaunchKernelGGL(k_cg_p, dim3(nb256(n)), dim3(256), 0, c->stream, n, z, p, sc);
    hipLaunchKernelGGL(k_shift, dim3(1), dim3(64), 0, c->stream, sc);
    return hipGetLastError();
}

int red_stage1_max() { return RED_MAX; }

namespace {
// out[blk] = sum of part[blk*chunk .. min(n, (blk+1)*chunk))
__global__ void __launch_bounds__(RT) k_chunk_sum(const double *__restrict__ part, int64_t n,
                                                  int64_t chunk, double *out)
{
    __shared__ double sh[RT / 64];
    const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += RT) s += part[i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}
}  // namespace

hipError_t reduce_parts(hx_ctx *c, const double *part, int64_t n, double *dst)
{
    if (n <= 8192) {
        // few partial sums: one workgroup, one launch
        hipLaunchKernelGGL(k_red2, dim3(1), dim3(RT), 0, c->stream, part, (int)n, 0, dst);
        return hipGetLastError();
    }
    const int64_t chunk = 4096;
    int64_t nb = (n + chunk - 1) / chunk;
    if (nb < 1) nb = 1;
    if (nb > RED_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_chunk_sum, dim3((unsigned)nb), dim3(RT), 0, c->stream, part, n, chunk, c->red);
    hipLaunchKernelGGL(k_red2, dim3(1), dim3(RT), 0, c->stream, c->red, (int)nb, RED_MAX, dst);
    return hipGetLastError();
}

// One fused CG step around the preconditioner pc (none, block Jacobi, the
// cell mass blocks, a diagonal kind, or the Chebyshev polynomial after the
// update): x += a p, r -= a q, z = M^{-1} r, sc[2] = r.z, sc[3] = r.r.
// npq > 0: p.q is the sum of the operator's npq partial sums in c->pqpart.
// lp (may be null): the loop's state; the step kernels read the current r.z
// from slot lp->cur of sc, and with p.q from the operator's partial sums,
// at most 8,192 partial sums of the step and a final z the sums are left to
// the direction update (CG_DEFERRED).
template <typename T>
hipError_t cg_step_pc(hx_ctx *c, int pc, T *x, T *r, const T *p, const T *q, T *z, double *sc_base,
                      double *host_rr, int *flags, int npq, CgLoop *lp)
{
    *flags = 0;
    const double *pqp = npq > 0 ? c->pqpart : nullptr;
    // the current r.z in sc[0] for the step kernels (slot 2 only ever with
    // p.q from partial sums, so the kernels do not read sc[1])
    double *sc = sc_base + (lp ? lp->cur : 0);
    const int64_t n = c->n_dofs;
    const int ld = (int)c->n_cells + 1;
    const bool dbl = sizeof(T) == 8;
    int nb = 0;
    hipError_t e;
    if (pc == HX_PC_BLOCK_JACOBI) {
        e = dbl ? launch_cg_bj64(c, (double *)x, (double *)r, (const double *)p, (const double *)q,
                                 (double *)z, sc, &nb, pqp, npq)
                : launch_cg_bj32(c, (float *)x, (float *)r, (const float *)p, (const float *)q,
                                 (float *)z, sc, &nb, pqp, npq);
    } else if (pc == HX_PC_MASS_BLOCK) {
        e = dbl ? launch_cg_massinv64(c, (double *)x, (double *)r, (const double *)p,
                                      (const double *)q, (double *)z, sc, &nb, pqp, npq)
                : launch_cg_massinv32(c, (float *)x, (float *)r, (const float *)p, (const float *)q,
                                      (float *)z, sc, &nb, pqp, npq);
    } else {
        const T *dinv = nullptr;
        if (pc == HX_PC_HELMHOLTZ_DIAG || pc == HX_PC_MASS_DIAG) {
            const int w = pc == HX_PC_HELMHOLTZ_DIAG ? 0 : 1;
            dinv = dbl ? (const T *)(c->dg64 + (int64_t)w * n) : (const T *)(c->dg32 + (int64_t)w * n);
        }
        nb = red_blocks(n);
        if (nb > ld) nb = ld;   // rows of c->cgpart (n_cells + 1 partial sums)
        // the FP32 V-cycle reads r rounded to FP32 from its level vector
        float *r32 = nullptr;
        if constexpr (sizeof(T) == 8)
            if (pc == HX_PC_MULTIGRID_MIXED) r32 = c->mgw32;
        hipLaunchKernelGGL(k_cg_elem<T>, dim3(nb), dim3(RT), 0, c->stream, n, x, r, p, q, z, dinv,
                           sc, c->cgpart, ld, r32, pqp, npq);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return e;
    const bool z_final = pc != HX_PC_CHEBYSHEV && pc != HX_PC_MULTIGRID && pc != HX_PC_MULTIGRID_MIXED;
    if (nb > 8192) {
        // one partial sum per block of the fused cell-block kernels: two stages
        e = reduce_parts(c, c->cgpart, nb, sc + 2);
        if (e == hipSuccess) e = reduce_parts(c, c->cgpart + ld, nb, sc + 3);
    } else if (z_final && lp && pqp) {
        // the direction update sums r.z and r.r itself
        lp->nb = nb;
        lp->host = host_rr;
        *flags = CG_DEFERRED | (host_rr ? CG_RR_ON_HOST : 0);
    } else if (z_final) {
        // the sums, the direction coefficient and r.r for the host in one launch
        hipLaunchKernelGGL(k_red_cg, dim3(2), dim3(RT), 0, c->stream, c->cgpart, nb, ld, sc, host_rr);
        e = hipGetLastError();
        *flags = CG_BETA_READY | (host_rr ? CG_RR_ON_HOST : 0);
    } else {
        hipLaunchKernelGGL(k_red2, dim3(2), dim3(RT), 0, c->stream, c->cgpart, nb, ld, sc + 2);
        e = hipGetLastError();
    }
    if constexpr (sizeof(T) == 8) {
        // the polynomial and multigrid preconditioners: z = r above, now
        // z = p(M^-1 A) M^-1 r or one V-cycle, and sc[2] = r.z
        if (e == hipSuccess && (pc == HX_PC_CHEBYSHEV || pc == HX_PC_MULTIGRID)) {
            e = pc == HX_PC_CHEBYSHEV ? cheb_apply64(c, (const double *)r, (double *)z)
                                      : mg_vcycle64(c, (const double *)r, (double *)z);
            if (e == hipSuccess) e = blas_dot(c, n, (const double *)r, (const double *)z, sc + 2);
        }
        if (e == hipSuccess && pc == HX_PC_MULTIGRID_MIXED) {
            // r in FP32 is already in place: the cycle, then z and r.z in one pass
            e = mg_vcycle32_resident(c);
            if (e == hipSuccess) {
                const int nbd = red_blocks(n);
                hipLaunchKernelGGL(k_widen_dot, dim3(nbd), dim3(RT), 0, c->stream, n,
                                   (const float *)(c->mgw32 + n), (const double *)r, (double *)z,
                                   c->red);
                hipLaunchKernelGGL(k_red2, dim3(1), dim3(RT), 0, c->stream, c->red, nbd, RED_MAX,
                                   sc + 2);
                e = hipGetLastError();
            }
        }
    }
    return e;
}

template <typename T>
hipError_t cg_step_p(hx_ctx *c, const T *z, T *p, double *sc, int flags, CgLoop *lp)
{
    const int64_t n = c->n_dofs;
    if (flags & CG_DEFERRED) {
        hipLaunchKernelGGL(k_cg_pt_red<T>, dim3(nb256(n)), dim3(256), 0, c->stream, n, z, p,
                           (const double *)c->cgpart, lp->nb, (int)c->n_cells + 1, sc, lp->cur,
                           lp->host);
        lp->cur = 2 - lp->cur;
        return hipGetLastError();
    }
    const int ready = (flags & CG_BETA_READY) ? 1 : 0;
    hipLaunchKernelGGL(k_cg_pt<T>, dim3(nb256(n)), dim3(256), 0, c->stream, n, z, p, sc, ready);
    if (!ready) hipLaunchKernelGGL(k_shift, dim3(1), dim3(64), 0, c->stream, sc);
    return hipGetLastError();
}

hipError_t cg_step_pc64(hx_ctx *c, int pc, double *x, double *r, const double *p, const double *q,
                        double *z, double *sc, double *host_rr, int *flags, int npq, CgLoop *lp)
{
    return cg_step_pc<double>(c, pc, x, r, p, q, z, sc, host_rr, flags, npq, lp);
}
hipError_t cg_step_pc32(hx_ctx *c, int pc, float *x, float *r, const float *p, const float *q,
                        float *z, double *sc, int *flags, int npq, CgLoop *lp)
{
    return cg_step_pc<float>(c, pc, x, r, p, q, z, sc, nullptr, flags, npq, lp);
}
hipError_t cg_step_p64(hx_ctx *c, const double *z, double *p, double *sc, int flags, CgLoop *lp)
{
    return cg_step_p<double>(c, z, p, sc, flags, lp);
}
hipError_t cg_step_p32(hx_ctx *c, const float *z, float *p, double *sc, int flags, CgLoop *lp)
{
    return cg_step_p<float>(c, z, p, sc, flags, lp);
}

}  // namespace hx
