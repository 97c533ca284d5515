// Learned per-cell preconditioner: feature gather, BF16 MFMA network
// forward/backward, Adam, and the correction added to block Jacobi.
//
// Network n_in -> 256 -> 256 -> n_out with ReLU, n_in = N^3 + 6 N^2 + 1,
// n_out = N^3.  Parameters flat [W1, b1, W2, b2, W3, b3], W row-major
// [out][in]; FP32 master weights and Adam moments, BF16 working copies.
// Every product runs on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16
// for the K-contiguous forward products, v_mfma_f32_16x16x16_bf16 for the
// strided ones of the backward pass; FP32 accumulation); activations entering a product are BF16 (round to
// nearest even), biases, losses and gradients of the biases are FP32.
//
// Features of cell K (divided by s = RMS(r_K), zero when s = 0): r_K in local
// order, then for each face -x,+x,-y,+y,-z,+z the neighbour's residual on its
// N^2 Gauss-Lobatto nodes of the shared face (tangential lexicographic order,
// lower direction fastest; zero on a boundary), then log(bbar/(abar l^2)).
// The correction added to block Jacobi is w_K net(features)_K with w_K the RMS
// of the block-Jacobi output on the cell, so the network works in O(1) units.
#include "common.hpp"
#include "bj_cell.hpp"
#include "sum256.hpp"

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

namespace hx {

namespace {

constexpr int HID = 256;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return 0x7FC0;   // NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// C(m, n) = sum_k A(m, k) B(n, k) (+ bias[n]) (ReLU), A(m,k) = A[m*sam + k*sak],
// B(n,k) = B[n*sbn + k*sbk], BF16 operands, FP32 accumulation on MFMA.
// 64 x 64 output tile per workgroup of 4 waves, 32 x 32 per wave.
// ---------------------------------------------------------------------------
constexpr int TM = 64, TN = 64, TK = 32;

__global__ void __launch_bounds__(256)
k_gemm(int M, int N, int K, const uint16_t *__restrict__ A, int64_t sam, int64_t sak,
       const uint16_t *__restrict__ B, int64_t sbn, int64_t sbk, const float *__restrict__ bias,
       int relu, float *C32, int64_t ldc32, uint16_t *C16, int64_t ldc16)
{
    __shared__ uint16_t sA[TM][TK + 4];
    __shared__ uint16_t sB[TN][TK + 4];
    const int m0 = blockIdx.x * TM, n0 = blockIdx.y * TN;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += TK) {
        // stage the tiles (zero outside the matrices)
        for (int e = t; e < TM * TK; e += 256) {
            const int r = e / TK, kk = e % TK;
            const int m = m0 + r, k = k0 + kk;
            sA[r][kk] = (m < M && k < K) ? A[(int64_t)m * sam + (int64_t)k * sak] : (uint16_t)0;
            const int n = n0 + r;
            sB[r][kk] = (n < N && k < K) ? B[(int64_t)n * sbn + (int64_t)k * sbk] : (uint16_t)0;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < TK; ks += 16) {
            // operand layout of the 16x16x16 MFMA: lane l holds
            //   A[row = l % 16][k = 4 (l / 16) .. +3],  B[k = 4 (l / 16) .. +3][col = l % 16]
            const int rr = lane & 15, kq = (lane >> 4) * 4;
            bf16x4 fa[2], fb[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    fa[i][q] = (short)sA[wm + 16 * i + rr][ks + kq + q];
                    fb[i][q] = (short)sB[wn + 16 * i + rr][ks + kq + q];
                }
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fa[i], fb[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    // result layout: lane l holds C[row = 4 (l / 16) + q][col = l % 16], q = 0..3
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
                const int n = n0 + wn + 16 * j + (lane & 15);
                if (m < M && n < N) {
                    float v = acc[i][j][q] + (bias ? bias[n] : 0.f);
                    if (relu) v = v > 0.f ? v : 0.f;
                    if (C32) C32[(int64_t)m * ldc32 + n] = v;
                    if (C16) C16[(int64_t)m * ldc16 + n] = f2bf(v);
                }
            }
}

// ---------------------------------------------------------------------------
// The same product when both operands are K-contiguous (A [M][K], B [N][K],
// K a multiple of 32, rows 16-byte aligned) -- every forward product of the
// network.  128 x 128 output tile per workgroup of 4 waves (64 x 64 each, a
// 4 x 4 grid of 16 x 16 accumulators), 16-byte tile loads into padded LDS
// rows, v_mfma_f32_16x16x32_bf16 (gfx950): lane l supplies A[row l % 16] and
// B[col l % 16] at the same 8 consecutive k, 8 (l / 16) .. + 7, so the
// product pairs matching k whatever order the unit sums them in.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int NM = 128, NN = 128, NK = 32, NPAD = 8;

__global__ void __launch_bounds__(256)
k_gemm_nt(int M, int N, int K, const uint16_t *__restrict__ A, int64_t lda,
          const uint16_t *__restrict__ B, int64_t ldb, const float *__restrict__ bias, int relu,
          float *C32, int64_t ldc32, uint16_t *C16, int64_t ldc16)
{
    __shared__ __attribute__((aligned(16))) uint16_t sA[NM][NK + NPAD];
    __shared__ __attribute__((aligned(16))) uint16_t sB[NN][NK + NPAD];
    const int m0 = blockIdx.x * NM, n0 = blockIdx.y * NN;
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int wm = (wave & 1) * 64, wn = (wave >> 1) * 64;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const uint4 zero = {0u, 0u, 0u, 0u};
    for (int k0 = 0; k0 < K; k0 += NK) {
        // 128 rows x 32 k per operand = 512 chunks of 8 values, 2 per thread
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ch = t + 256 * h, row = ch >> 2, kc = (ch & 3) * 8;
            const int m = m0 + row, n = n0 + row;
            const uint4 va = m < M ? *(const uint4 *)(A + (int64_t)m * lda + k0 + kc) : zero;
            const uint4 vb = n < N ? *(const uint4 *)(B + (int64_t)n * ldb + k0 + kc) : zero;
            *(uint4 *)&sA[row][kc] = va;
            *(uint4 *)&sB[row][kc] = vb;
        }
        __syncthreads();
        const int rr = lane & 15, kq = (lane >> 4) * 8;
        bf16x8 fa[4], fb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            fa[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)&sA[wm + 16 * i + rr][kq]);
            fb[i] = __builtin_bit_cast(bf16x8, *(const uint4 *)&sB[wn + 16 * i + rr][kq]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // result layout: lane l holds C[row = 4 (l / 16) + q][col = l % 16], q = 0..3
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int n = n0 + wn + 16 * j + (lane & 15);
            const float bn = (bias && n < N) ? bias[n] : 0.f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
                if (m < M && n < N) {
                    float v = acc[i][j][q] + bn;
                    if (relu) v = v > 0.f ? v : 0.f;
                    if (C32) C32[(int64_t)m * ldc32 + n] = v;
                    if (C16) C16[(int64_t)m * ldc16 + n] = f2bf(v);
                }
            }
        }
}

hipError_t gemm(hipStream_t st, int M, int N, int K, const uint16_t *A, int64_t sam, int64_t sak,
                const uint16_t *B, int64_t sbn, int64_t sbk, const float *bias, int relu, float *C32,
                int64_t ldc32, uint16_t *C16, int64_t ldc16)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    if (sak == 1 && sbk == 1 && K % NK == 0 && sam % 8 == 0 && sbn % 8 == 0 &&
        ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0) {
        dim3 grid((M + NM - 1) / NM, (N + NN - 1) / NN);
        hipLaunchKernelGGL(k_gemm_nt, grid, dim3(256), 0, st, M, N, K, A, sam, B, sbn, bias, relu,
                           C32, ldc32, C16, ldc16);
        return hipGetLastError();
    }
    dim3 grid((M + TM - 1) / TM, (N + TN - 1) / TN);
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, M, N, K, A, sam, sak, B, sbn, sbk, bias, relu,
                       C32, ldc32, C16, ldc16);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise / reduction kernels
// ---------------------------------------------------------------------------
__global__ void k_weights_to_bf16(int64_t n, const float *__restrict__ w, int rows, int cols,
                                  int ld, uint16_t *out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)rows * ld) return;
    const int r = (int)(i / ld), c = (int)(i % ld);
    out[i] = c < cols ? f2bf(w[(int64_t)r * cols + c]) : (uint16_t)0;
    (void)n;
}

// fp32 [rows][cols] -> bf16 in the fused kernel's fragment order: for
// column tile ct (16 output columns), k-step s (32 inputs) and lane l the
// 8 values W[16 ct + l % 16][32 s + 8 (l / 16) .. + 7] sit at
// ((ct ks + s) 64 + l) 8, so that one wave's fragment load is 1 KB in a
// row and its whole slice of a layer is contiguous; rows past rows and
// inputs past cols are zero
__global__ void k_weights_frag(const float *__restrict__ w, int rows, int cols, int ks, uint16_t *out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= (int64_t)((rows + 15) / 16) * ks * 512) return;
    const int e = (int)(i & 7), lane = (int)((i >> 3) & 63);
    const int64_t blk = i >> 9;
    const int s = (int)(blk % ks), ct = (int)(blk / ks);
    const int r = ct * 16 + (lane & 15), k = s * 32 + (lane >> 4) * 8 + e;
    out[i] = (r < rows && k < cols) ? f2bf(w[(int64_t)r * cols + k]) : (uint16_t)0;
}

// fp32 [B][n_in] -> bf16 [B][ld]
__global__ void k_pack(int64_t Bn, int n_in, int ld, const float *__restrict__ x, uint16_t *out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= Bn * ld) return;
    const int64_t r = i / ld;
    const int c = (int)(i % ld);
    out[i] = c < n_in ? f2bf(x[r * n_in + c]) : (uint16_t)0;
}

// features: block per cell
__global__ void __launch_bounds__(128)
k_features(int n, int64_t n_cells, const double *__restrict__ r, const int32_t *__restrict__ nbr,
           const double *__restrict__ coef, float *feats, int64_t ldf, uint16_t *fb, int64_t ldb,
           float *scale)
{
    const int64_t c = blockIdx.x;
    const int nd = n * n * n, nf = n * n;
    const int n_in = nd + 6 * nf + 1;
    __shared__ double red[128];
    double ss = 0.0;
    for (int e = threadIdx.x; e < nd; e += 128) {
        const double v = r[c * nd + e];
        ss += v * v;
    }
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int s = 64; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double sK = sqrt(red[0] / nd);
    const double inv = sK > 0.0 ? 1.0 / sK : 0.0;
    for (int e = threadIdx.x; e < n_in; e += 128) {
        double v = 0.0;
        if (e < nd) {
            v = r[c * nd + e] * inv;
        } else if (e < nd + 6 * nf) {
            const int f = (e - nd) / nf, t = (e - nd) % nf;
            const int32_t nb = nbr[c * 6 + f];
            if (nb >= 0) {
                const int d = f >> 1, plus = f & 1;
                const int m = plus ? 0 : n - 1;     // the neighbour's layer touching the face
                const int p = t % n, q = t / n;      // tangential, lower direction fastest
                int ijk[3];
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                ijk[d] = m;
                ijk[t1] = p;
                ijk[t2] = q;
                v = r[(int64_t)nb * nd + ijk[0] + n * (ijk[1] + n * ijk[2])] * inv;
            }
        } else {
            v = sK > 0.0 ? coef[c] : 0.0;
        }
        const float fv = (float)v;
        if (feats) feats[c * ldf + e] = fv;
        if (fb) fb[c * ldb + e] = f2bf(fv);
    }
    if (fb)
        for (int e = n_in + threadIdx.x; e < ldb; e += 128) fb[c * ldb + e] = 0;
    if (threadIdx.x == 0) scale[c] = (float)sK;
}

// d_o = 2 (o - t) / (B n_out) (fp32 and bf16); partial sums of (o - t)^2
__global__ void __launch_bounds__(256)
k_loss_grad(int64_t total, float inv_count, const float *__restrict__ o, const float *__restrict__ tg,
            float *d, uint16_t *db, double *part)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const float e = o[i] - tg[i];
        s += (double)e * e;
        const float g = 2.f * e * inv_count;
        d[i] = g;
        db[i] = f2bf(g);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_sum_parts(int nb, const double *part, double scale, float *out)
{
    __shared__ double sh[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = (float)(sh[0] * scale);
}

// d[b][j] *= (h[b][j] > 0) in place (fp32), bf16 copy
__global__ void k_relu_back(int64_t total, const float *__restrict__ h, float *d, uint16_t *db)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= total) return;
    const float g = h[i] > 0.f ? d[i] : 0.f;
    d[i] = g;
    db[i] = f2bf(g);
}

// column sums out[j] = sum_b d[b][j] (fixed order), block per column
__global__ void __launch_bounds__(256) k_colsum(int64_t Bn, int ncol, const float *__restrict__ d, float *out)
{
    __shared__ double sh[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int64_t b = threadIdx.x; b < Bn; b += 256) s += d[b * ncol + j];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = (float)sh[0];
}

__global__ void k_adam(int64_t n, float *w, const float *__restrict__ g, float *m, float *v, float lr,
                       float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// per cell w_K = RMS(z_K) of the block-Jacobi output; z_K += w_K * o_K
__global__ void __launch_bounds__(128)
k_add_correction(int nd, const float *__restrict__ o, double *z)
{
    const int64_t c = blockIdx.x;
    __shared__ double red[128];
    double ss = 0.0;
    for (int e = threadIdx.x; e < nd; e += 128) {
        const double v = z[c * nd + e];
        ss += v * v;
    }
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int k = 64; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double w = sqrt(red[0] / nd);
    for (int e = threadIdx.x; e < nd; e += 128) z[c * nd + e] += w * (double)o[c * nd + e];
}

// ---------------------------------------------------------------------------
// The learned preconditioner, a workgroup of FW waves serving 16 cells.  It
// reads r_K (WBJ: scaled by s = 1/|w| when the partial sums of |w|^2 are
// given, the normalisation of the Krylov vector, whose result it also
// writes), forms the features (as k_features: r_K, the six neighbours' face
// layers and the coefficient feature, scaled by 1 / RMS(r_K)) in LDS as BF16,
// obtains BJ(r)_K (WBJ: solves the cells' block-Jacobi systems in LDS with
// the sweeps of the block-Jacobi kernels, so the whole preconditioner is one
// launch; otherwise reads it from z, written by the block-Jacobi kernel),
// runs the three layers on v_mfma_f32_16x16x32_bf16 with the hidden
// activations in LDS (each wave owns a share of every layer's outputs and
// loads the weight fragments of several k-steps at once, so their latency
// is paid once per chunk), and writes z_K = BJ(r)_K + w_K net(features)_K
// with w_K = RMS(BJ(r)_K).
// Fragment layout of the MFMA: lane l holds A[m = l % 16][k = 8 (l / 16) ..
// + 7] and B[k][n = l % 16] likewise, and receives C[4 (l / 16) + q][l % 16].
constexpr int FT = 16;   // cells per workgroup of the fused kernel

// One wave's weight fragments of its NT column tiles over all KS k-steps
// from a layer in fragment order (n_tiles column tiles), issued together
// without branches: a tile at or past n_tiles reads the last one (its
// results are never stored)
template <int KS, int NT>
__device__ __forceinline__ void layer_weights(const uint16_t *__restrict__ P, int n_tiles, int ct0,
                                              int lane, uint4 (&fb)[KS][NT])
{
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int ct = min(ct0 + j, n_tiles - 1);
            fb[s][j] = *(const uint4 *)(P + ((int64_t)(ct * KS + s) * 64 + lane) * 8);
        }
    }
}

// acc[j] = (16 rows of sA) x (column tile j of the weights in fb)
template <int K, int NT, int LDA>
__device__ __forceinline__ void layer_mfma(const uint16_t (*sA)[LDA], const uint4 (&fb)[K / 32][NT],
                                           int lane, f32x4 (&acc)[NT])
{
    const int rr = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < K / 32; ++s) {
        const bf16x8 fa = __builtin_bit_cast(bf16x8, *(const uint4 *)&sA[rr][s * 32 + kq]);
#pragma unroll
        for (int j = 0; j < NT; ++j)
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, __builtin_bit_cast(bf16x8, fb[s][j]),
                                                             acc[j], 0, 0, 0);
    }
}

constexpr int FW = 16;   // waves per workgroup of the fused kernel

// offset inside the neighbour cell of face feature t of face f (the
// neighbour's touching layer, tangential lexicographic order, lower
// direction fastest), for every f * N^2 + t
template <int N>
struct FaceFeat {
    int off[6 * N * N];
    constexpr FaceFeat() : off()
    {
        for (int f = 0; f < 6; ++f)
            for (int t = 0; t < N * N; ++t) {
                const int d = f >> 1, m = (f & 1) ? 0 : N - 1;
                int ijk[3] = {0, 0, 0};
                ijk[d] = m;
                ijk[d == 0 ? 1 : 0] = t % N;
                ijk[d == 2 ? 1 : 2] = t / N;
                off[f * N * N + t] = ijk[0] + N * (ijk[1] + N * ijk[2]);
            }
    }
};
template <int N>
__device__ constexpr FaceFeat<N> kFaceFeat{};

template <int N, bool WBJ>
__global__ void __launch_bounds__(64 * FW)
k_mlp_fused(int64_t n_cells, const double *__restrict__ w, double *__restrict__ z,
            const int32_t *__restrict__ nbr, const double *__restrict__ coef,
            const uint16_t *__restrict__ wfr, const float *__restrict__ b1, const float *__restrict__ b2,
            const float *__restrict__ b3, const double *__restrict__ bjS,
            const double *__restrict__ bjL, const double *__restrict__ bjC,
            const double *__restrict__ part, int nbp, double *__restrict__ vout)
{
    constexpr int NF = N * N, ND = NF * N, NIN = ND + 6 * NF + 1, LDX = ((NIN + 31) / 32) * 32;
    constexpr int NTH = 64 * FW, PER = (HID / 16) / FW;   // column tiles of 16 per wave, hidden layers
    constexpr int NT3 = (ND + 15) / 16, PER3 = (NT3 + FW - 1) / FW;
    constexpr int SUB = NTH / FT;                         // threads per cell in the norms
    static_assert(PER * FW * 16 == HID && SUB >= 16 && (SUB & (SUB - 1)) == 0, "layout");
    static_assert(FT * NF <= NTH && NTH >= 256, "block-Jacobi threads");
    constexpr int FB = WBJ ? FT : 1;
    __shared__ __align__(16) uint16_t sX[FT][LDX + 8];
    __shared__ __align__(16) uint16_t sH[FT][HID + 8];
    __shared__ __align__(16) uint16_t sH2[FT][HID + 8];
    __shared__ double sR[FT][ND];          // r_K, then BJ(r)_K
    __shared__ double sBS[FB][3][NF], sBL[FB][3][N], sBC[FB][4];
    __shared__ double sS[FT], sInv[FT], sW[FT], sCf[FT], sh4[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t c0 = (int64_t)blockIdx.x * FT;
    constexpr int RPT = (ND + SUB - 1) / SUB;            // own values per thread
    constexpr int FPT = (FT * LDX + NTH - 1) / NTH;      // feature slots per thread
    constexpr int SPT = (FT * 3 * NF + NTH - 1) / NTH;   // eigenvector entries per thread
    constexpr int LPT = (FT * 3 * N + NTH - 1) / NTH;    // eigenvalues per thread
    constexpr int ZPT = (FT * ND + NTH - 1) / NTH;       // block-Jacobi outputs per thread
    const int cl_r = tid / SUB, sub = tid % SUB;
    const bool own_ok = c0 + cl_r < n_cells;
    // First batch of loads, all in flight together with the partial sums of
    // the scale below (every address valid; an unused entry reads element
    // 0): the own values, the neighbour index and the coefficient feature of
    // each of this thread's feature slots, the block-Jacobi tables.
    double wv[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int e = sub + u * SUB;
        wv[u] = w[(own_ok && e < ND) ? (c0 + cl_r) * ND + e : 0];
    }
    int32_t fnb[FPT], foff[FPT];
#pragma unroll
    for (int u = 0; u < FPT; ++u) {
        const int idx = tid + u * NTH, cl = idx / LDX, e = idx % LDX;
        const int64_t c = c0 + cl;
        const bool isn = idx < FT * LDX && c < n_cells && e >= ND && e < ND + 6 * NF;
        const int32_t nbv = nbr[isn ? c * 6 + (e - ND) / NF : 0];
        fnb[u] = isn ? nbv : -1;
        foff[u] = kFaceFeat<N>.off[isn ? e - ND : 0];
    }
    const double cfv = coef[(tid < FT && c0 + tid < n_cells) ? c0 + tid : 0];
    double tS[SPT], tL[LPT], tC = 0.0;
    if constexpr (WBJ) {
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int idx = tid + u * NTH, cl = idx / (3 * NF);
            const bool ok = idx < FT * 3 * NF && c0 + cl < n_cells;
            tS[u] = bjS[ok ? (c0 + cl) * 3 * NF + idx % (3 * NF) : 0];
        }
#pragma unroll
        for (int u = 0; u < LPT; ++u) {
            const int idx = tid + u * NTH, cl = idx / (3 * N);
            const bool ok = idx < FT * 3 * N && c0 + cl < n_cells;
            tL[u] = bjL[ok ? (c0 + cl) * 3 * N + idx % (3 * N) : 0];
        }
        tC = bjC[(tid < FT * 4 && c0 + tid / 4 < n_cells) ? (c0 + tid / 4) * 4 + tid % 4 : 0];
    }
    // the Krylov vector's scale (the fixed-order sum the host repeats)
    const double sc = part ? 1.0 / sqrt(sum256(part, nbp, sh4)) : 1.0;
    // second batch: the neighbours' face-layer values of the feature slots
    // and, without the block-Jacobi solve here, the block-Jacobi output
    double fval[FPT];
#pragma unroll
    for (int u = 0; u < FPT; ++u) {
        const int32_t nb = fnb[u];
        int64_t a = 0;
        if (nb >= 0) a = (int64_t)nb * ND + foff[u];
        fval[u] = w[a];
    }
    double zv[ZPT];
    if constexpr (!WBJ) {
#pragma unroll
        for (int u = 0; u < ZPT; ++u) {
            const int idx = tid + u * NTH, cl = idx / ND;
            zv[u] = z[(idx < FT * ND && c0 + cl < n_cells) ? (c0 + cl) * ND + idx % ND : 0];
        }
    }
    // r_K = sc w_K into LDS (and to vout), its RMS: SUB threads per cell
    {
        double sr = 0.0;
        if (own_ok) {
#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int e = sub + u * SUB;
                if (e < ND) {
                    const double v = wv[u] * sc;
                    sR[cl_r][e] = v;
                    if (vout) vout[(c0 + cl_r) * ND + e] = v;
                    sr += v * v;
                }
            }
        }
#pragma unroll
        for (int o = SUB / 2; o > 0; o >>= 1) sr += __shfl_xor(sr, o, 64);
        if (sub == 0) {
            const double sK = sqrt(sr / ND);
            sS[cl_r] = sK;
            sInv[cl_r] = sK > 0.0 ? 1.0 / sK : 0.0;
        }
    }
    if (tid < FT) sCf[tid] = cfv;
    // block-Jacobi tables of the workgroup's cells
    if constexpr (WBJ) {
#pragma unroll
        for (int u = 0; u < SPT; ++u) {
            const int idx = tid + u * NTH, cl = idx / (3 * NF), e = idx % (3 * NF);
            if (idx < FT * 3 * NF && c0 + cl < n_cells) sBS[cl][e / NF][e % NF] = tS[u];
        }
#pragma unroll
        for (int u = 0; u < LPT; ++u) {
            const int idx = tid + u * NTH, cl = idx / (3 * N), e = idx % (3 * N);
            if (idx < FT * 3 * N && c0 + cl < n_cells) sBL[cl][e / N][e % N] = tL[u];
        }
        if (tid < FT * 4 && c0 + tid / 4 < n_cells) sBC[tid / 4][tid % 4] = tC;
    }
    __syncthreads();
    // features, BF16
#pragma unroll
    for (int u = 0; u < FPT; ++u) {
        const int idx = tid + u * NTH;
        if (idx >= FT * LDX) break;
        const int cl = idx / LDX, e = idx % LDX;
        const int64_t c = c0 + cl;
        float fv = 0.f;
        if (c < n_cells && e < NIN) {
            const double sK = sS[cl], inv = sInv[cl];
            double v = 0.0;
            if (e < ND) {
                v = sR[cl][e] * inv;
            } else if (e < ND + 6 * NF) {
                if (fnb[u] >= 0) v = (fval[u] * sc) * inv;
            } else {
                v = sK > 0.0 ? sCf[cl] : 0.0;
            }
            fv = (float)v;
        }
        sX[cl][e] = f2bf(fv);
    }
    if constexpr (WBJ) {
        // block Jacobi in place: NF threads per cell
        const int lc0 = tid / NF, lc = lc0 < FT ? lc0 : 0, tt = tid - lc0 * NF;
        const bool active = lc0 < FT && c0 + lc0 < n_cells;
        double unused = 0.0;
        bj_cell_solve<N, double>(sR[lc], sBS[lc], sBL[lc], sBC[lc], tt % N, tt / N, active, unused);
    } else {
        // BJ(r) from z (loaded above), once the features have read r
        __syncthreads();
#pragma unroll
        for (int u = 0; u < ZPT; ++u) {
            const int idx = tid + u * NTH, cl = idx / ND;
            if (idx < FT * ND && c0 + cl < n_cells) sR[cl][idx % ND] = zv[u];
        }
        __syncthreads();
    }
    // Weight fragments.  The one-launch form (at most one workgroup per
    // compute unit, so its register count costs no occupancy) loads them a
    // layer ahead: layers 1 and 2 here, in flight during the norms below,
    // layer 3 once layer 1's products are issued.  The other form loads
    // each layer's just before its products (two workgroups per compute
    // unit at the smaller degrees).
    // The biases of the lane's output columns come first, so that waiting
    // for them never waits for weights issued later.
    constexpr int KS1 = LDX / 32, KS2 = HID / 32;
    const uint16_t *__restrict__ w1f = wfr;
    const uint16_t *__restrict__ w2f = wfr + (HID / 16) * KS1 * 512;
    const uint16_t *__restrict__ w3f = w2f + (HID / 16) * KS2 * 512;
    uint4 f1[KS1][PER], f2[KS2][PER], f3[KS2][PER3];
    float bv1[PER], bv2[PER], bv3[PER3];
    const int ccol = lane & 15, crow = 4 * (lane >> 4);
    auto biases = [&](const float *__restrict__ bsrc, int n_rows, int per, float *bv) {
        for (int j = 0; j < per; ++j) {
            const int n = (per * wave + j) * 16 + ccol;
            bv[j] = bsrc[n < n_rows ? n : 0];
        }
    };
    if constexpr (WBJ) {
        biases(b1, HID, PER, bv1);
        biases(b2, HID, PER, bv2);
        biases(b3, ND, PER3, bv3);
        layer_weights<KS1, PER>(w1f, HID / 16, PER * wave, lane, f1);
        layer_weights<KS2, PER>(w2f, HID / 16, PER * wave, lane, f2);
    }
    // w_K = RMS(BJ(r)_K)
    {
        const int cl = tid / SUB, sub = tid % SUB;
        double sz = 0.0;
        if (c0 + cl < n_cells)
            for (int e = sub; e < ND; e += SUB) sz += sR[cl][e] * sR[cl][e];
#pragma unroll
        for (int o = SUB / 2; o > 0; o >>= 1) sz += __shfl_xor(sz, o, 64);
        if (sub == 0) sW[cl] = sqrt(sz / ND);
    }
    // layer 1: each wave PER of the 16 column tiles (sX is complete: a
    // barrier follows the block-Jacobi step)
    {
        f32x4 acc[PER];
        if constexpr (!WBJ) {
            biases(b1, HID, PER, bv1);
            layer_weights<KS1, PER>(w1f, HID / 16, PER * wave, lane, f1);
        }
        layer_mfma<LDX, PER, LDX + 8>(sX, f1, lane, acc);
        if constexpr (WBJ) layer_weights<KS2, PER3>(w3f, NT3, PER3 * wave, lane, f3);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int n = (PER * wave + j) * 16 + ccol;
#pragma unroll
            for (int q = 0; q < 4; ++q) sH[crow + q][n] = f2bf(fmaxf(acc[j][q] + bv1[j], 0.f));
        }
    }
    __syncthreads();
    // layer 2
    {
        f32x4 acc[PER];
        if constexpr (!WBJ) {
            biases(b2, HID, PER, bv2);
            layer_weights<KS2, PER>(w2f, HID / 16, PER * wave, lane, f2);
        }
        layer_mfma<HID, PER, HID + 8>(sH, f2, lane, acc);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int n = (PER * wave + j) * 16 + ccol;
#pragma unroll
            for (int q = 0; q < 4; ++q) sH2[crow + q][n] = f2bf(fmaxf(acc[j][q] + bv2[j], 0.f));
        }
    }
    __syncthreads();
    // layer 3 and z = BJ(r) + w_K o_K
    {
        f32x4 acc[PER3];
        if constexpr (!WBJ) {
            biases(b3, ND, PER3, bv3);
            layer_weights<KS2, PER3>(w3f, NT3, PER3 * wave, lane, f3);
        }
        layer_mfma<HID, PER3, HID + 8>(sH2, f3, lane, acc);
#pragma unroll
        for (int j = 0; j < PER3; ++j) {
            const int n = (PER3 * wave + j) * 16 + ccol;
            if (n >= ND) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t c = c0 + crow + q;
                if (c < n_cells)
                    z[c * ND + n] = sR[crow + q][n] + sW[crow + q] * (double)(acc[j][q] + bv3[j]);
            }
        }
    }
}

// targets[c][i] = (e[c][i] - z[c][i]) / w_c with e = xs - xj, w_c = RMS(z_c)
// (0 when w_c = 0), limited to [-clip, clip] when clip > 0
__global__ void __launch_bounds__(128)
k_targets(int nd, const double *__restrict__ xs, const double *__restrict__ xj,
          const double *__restrict__ z, float clip, float *tg)
{
    const int64_t c = blockIdx.x;
    __shared__ double red[128];
    double ss = 0.0;
    for (int e = threadIdx.x; e < nd; e += 128) {
        const double v = z[c * nd + e];
        ss += v * v;
    }
    red[threadIdx.x] = ss;
    __syncthreads();
    for (int k = 64; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double w = sqrt(red[0] / nd);
    const double inv = w > 0.0 ? 1.0 / w : 0.0;
    for (int e = threadIdx.x; e < nd; e += 128) {
        const int64_t i = c * nd + e;
        float t = (float)((xs[i] - xj[i] - z[i]) * inv);
        if (clip > 0.f) t = fminf(fmaxf(t, -clip), clip);
        tg[i] = t;
    }
}

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct MlpState {
    int n_in = 0, ldx = 0, n_out = 0;
    int64_t P = 0;
    int64_t off_w1 = 0, off_b1 = 0, off_w2 = 0, off_b2 = 0, off_w3 = 0, off_b3 = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint16_t *w1b = nullptr, *w2b = nullptr, *w3b = nullptr;
    uint16_t *wfr = nullptr;   // the three layers in the fused kernel's fragment order
    int64_t t = 0;
    int64_t cap = 0;
    int64_t trace_B = 0;     // batch of the last training step whose buffers are intact
    uint16_t *xb = nullptr, *h1b = nullptr, *h2b = nullptr, *dob = nullptr, *dh1b = nullptr,
             *dh2b = nullptr;
    float *h1 = nullptr, *h2 = nullptr, *o = nullptr, *d_o = nullptr, *dh1 = nullptr,
          *dh2 = nullptr, *scale = nullptr, *loss = nullptr;
    double *part = nullptr, *zt = nullptr;
    float *loss_host = nullptr;
    int n_cu = 0;            // compute units of the device
};

static void free_batch(MlpState *s)
{
    void **b[] = {(void **)&s->xb, (void **)&s->h1b, (void **)&s->h2b, (void **)&s->dob,
                  (void **)&s->dh1b, (void **)&s->dh2b, (void **)&s->h1, (void **)&s->h2,
                  (void **)&s->o, (void **)&s->d_o, (void **)&s->dh1, (void **)&s->dh2,
                  (void **)&s->scale};
    for (void **p : b) dfree(p);
    s->cap = 0;
}

static hx_status ensure_batch(hx_ctx *c, int64_t B)
{
    MlpState *s = c->mlp;
    s->trace_B = 0;
    if (B <= s->cap) return HX_OK;
    free_batch(s);
    hx_status st = HX_OK;
#define A(p, bytes) \
    if (st == HX_OK) st = dalloc(c, (void **)&(p), (bytes));
    A(s->xb, 2 * (size_t)B * s->ldx);
    A(s->h1b, 2 * (size_t)B * HID);
    A(s->h2b, 2 * (size_t)B * HID);
    A(s->dob, 2 * (size_t)B * s->n_out);
    A(s->dh1b, 2 * (size_t)B * HID);
    A(s->dh2b, 2 * (size_t)B * HID);
    A(s->h1, 4 * (size_t)B * HID);
    A(s->h2, 4 * (size_t)B * HID);
    A(s->o, 4 * (size_t)B * s->n_out);
    A(s->d_o, 4 * (size_t)B * s->n_out);
    A(s->dh1, 4 * (size_t)B * HID);
    A(s->dh2, 4 * (size_t)B * HID);
    A(s->scale, 4 * (size_t)B);
#undef A
    if (st != HX_OK) {
        free_batch(s);
        return st;
    }
    s->cap = B;
    return HX_OK;
}

int64_t mlp_param_count(const hx_ctx *c)
{
    const int64_t ni = c->nd + 6 * c->nf + 1, no = c->nd;
    return HID * ni + HID + HID * HID + HID + no * HID + no;
}

hx_status mlp_create(hx_ctx *c)
{
    if (c->mlp) return HX_OK;
    MlpState *s = new MlpState();
    c->mlp = s;
    s->n_in = c->nd + 6 * c->nf + 1;
    s->ldx = ((s->n_in + 31) / 32) * 32;
    s->n_out = c->nd;
    s->P = mlp_param_count(c);
    s->off_w1 = 0;
    s->off_b1 = s->off_w1 + (int64_t)HID * s->n_in;
    s->off_w2 = s->off_b1 + HID;
    s->off_b2 = s->off_w2 + (int64_t)HID * HID;
    s->off_w3 = s->off_b2 + HID;
    s->off_b3 = s->off_w3 + (int64_t)s->n_out * HID;
    hx_status st = HX_OK;
#define A(p, bytes) \
    if (st == HX_OK) st = dalloc(c, (void **)&(p), (bytes));
    A(s->w, 4 * (size_t)s->P);
    A(s->m, 4 * (size_t)s->P);
    A(s->v, 4 * (size_t)s->P);
    A(s->grad, 4 * (size_t)s->P);
    A(s->w1b, 2 * (size_t)HID * s->ldx);
    A(s->w2b, 2 * (size_t)HID * HID);
    A(s->w3b, 2 * (size_t)s->n_out * HID);
    A(s->wfr, 2 * (size_t)512 * ((HID / 16) * (s->ldx / 32) + (HID / 16) * (HID / 32) +
                                 ((s->n_out + 15) / 16) * (HID / 32)));
    A(s->part, 8 * 1024);
    A(s->loss, 16);
#undef A
    if (st == HX_OK && hipHostMalloc((void **)&s->loss_host, 16) != hipSuccess) st = HX_ERR_DEVICE;
    if (st == HX_OK &&
        hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
        st = HX_ERR_DEVICE;
    if (st != HX_OK) {
        mlp_destroy(c);
        return st;
    }
    return HX_OK;
}

void mlp_destroy(hx_ctx *c)
{
    MlpState *s = c->mlp;
    if (!s) return;
    free_batch(s);
    void **b[] = {(void **)&s->w, (void **)&s->m, (void **)&s->v, (void **)&s->grad,
                  (void **)&s->w1b, (void **)&s->w2b, (void **)&s->w3b, (void **)&s->wfr, (void **)&s->part,
                  (void **)&s->loss, (void **)&s->zt};
    for (void **p : b) dfree(p);
    if (s->loss_host) (void)hipHostFree(s->loss_host);
    delete s;
    c->mlp = nullptr;
}

static hipError_t refresh_bf16(hx_ctx *c)
{
    MlpState *s = c->mlp;
    hipLaunchKernelGGL(k_weights_to_bf16, dim3(nb256((int64_t)HID * s->ldx)), dim3(256), 0, c->stream,
                       s->P, s->w + s->off_w1, HID, s->n_in, s->ldx, s->w1b);
    hipLaunchKernelGGL(k_weights_to_bf16, dim3(nb256((int64_t)HID * HID)), dim3(256), 0, c->stream,
                       s->P, s->w + s->off_w2, HID, HID, HID, s->w2b);
    hipLaunchKernelGGL(k_weights_to_bf16, dim3(nb256((int64_t)s->n_out * HID)), dim3(256), 0,
                       c->stream, s->P, s->w + s->off_w3, s->n_out, HID, HID, s->w3b);
    const int ks1 = s->ldx / 32, ks = HID / 32;
    uint16_t *f2 = s->wfr + (int64_t)512 * (HID / 16) * ks1, *f3 = f2 + (int64_t)512 * (HID / 16) * ks;
    hipLaunchKernelGGL(k_weights_frag, dim3(nb256((int64_t)512 * (HID / 16) * ks1)), dim3(256), 0,
                       c->stream, s->w + s->off_w1, HID, s->n_in, ks1, s->wfr);
    hipLaunchKernelGGL(k_weights_frag, dim3(nb256((int64_t)512 * (HID / 16) * ks)), dim3(256), 0,
                       c->stream, s->w + s->off_w2, HID, HID, ks, f2);
    hipLaunchKernelGGL(k_weights_frag, dim3(nb256((int64_t)512 * ((s->n_out + 15) / 16) * ks)),
                       dim3(256), 0, c->stream, s->w + s->off_w3, s->n_out, HID, ks, f3);
    return hipGetLastError();
}

hx_status mlp_set(hx_ctx *c, const float *w, int64_t n)
{
    if (n != mlp_param_count(c))
        return fail(c, HX_ERR_ARG, "network has %lld parameters, got %lld",
                    (long long)mlp_param_count(c), (long long)n);
    hx_status st = mlp_create(c);
    if (st != HX_OK) return st;
    MlpState *s = c->mlp;
    HX_HIP(c, hipMemcpyAsync(s->w, w, 4 * (size_t)n, hipMemcpyHostToDevice, c->stream));
    HX_HIP(c, hipMemsetAsync(s->m, 0, 4 * (size_t)n, c->stream));
    HX_HIP(c, hipMemsetAsync(s->v, 0, 4 * (size_t)n, c->stream));
    s->t = 0;
    HX_HIP(c, refresh_bf16(c));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    return HX_OK;
}

hx_status mlp_get(const hx_ctx *cc, float *w, int64_t n)
{
    hx_ctx *c = const_cast<hx_ctx *>(cc);
    if (!c->mlp) return fail(c, HX_ERR_STATE, "no network loaded");
    if (n != c->mlp->P) return fail(c, HX_ERR_ARG, "size mismatch");
    HX_HIP(c, hipMemcpyAsync(w, c->mlp->w, 4 * (size_t)n, hipMemcpyDeviceToHost, c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    return HX_OK;
}

hx_status mlp_features(hx_ctx *c, const double *r, float *feats, float *scale)
{
    const int n_in = c->nd + 6 * c->nf + 1;
    hipLaunchKernelGGL(k_features, dim3((unsigned)c->n_cells), dim3(128), 0, c->stream, c->n,
                       c->n_cells, r, c->nbr, c->coef_feat, feats, (int64_t)n_in, (uint16_t *)nullptr,
                       (int64_t)0, scale);
    HX_HIP(c, hipGetLastError());
    return HX_OK;
}

// forward on the packed batch s->xb (B rows); h1/h2 bf16 (and fp32 for the
// backward pass when training), o fp32
static hipError_t forward_packed(hx_ctx *c, int64_t B, bool training)
{
    MlpState *s = c->mlp;
    hipError_t e;
    e = gemm(c->stream, (int)B, HID, s->ldx, s->xb, s->ldx, 1, s->w1b, s->ldx, 1, s->w + s->off_b1, 1,
             training ? s->h1 : nullptr, HID, s->h1b, HID);
    if (e != hipSuccess) return e;
    e = gemm(c->stream, (int)B, HID, HID, s->h1b, HID, 1, s->w2b, HID, 1, s->w + s->off_b2, 1,
             training ? s->h2 : nullptr, HID, s->h2b, HID);
    if (e != hipSuccess) return e;
    return gemm(c->stream, (int)B, s->n_out, HID, s->h2b, HID, 1, s->w3b, HID, 1, s->w + s->off_b3, 0,
                s->o, s->n_out, nullptr, 0);
}

hx_status mlp_forward(hx_ctx *c, const float *feats, int64_t B, float *out)
{
    if (!c->mlp) return fail(c, HX_ERR_STATE, "no network loaded");
    MlpState *s = c->mlp;
    hx_status st = ensure_batch(c, B);
    if (st != HX_OK) return st;
    hipLaunchKernelGGL(k_pack, dim3(nb256(B * s->ldx)), dim3(256), 0, c->stream, B, s->n_in, s->ldx,
                       feats, s->xb);
    HX_HIP(c, hipGetLastError());
    HX_HIP(c, forward_packed(c, B, false));
    HX_HIP(c, hipMemcpyAsync(out, s->o, 4 * (size_t)B * s->n_out, hipMemcpyDeviceToDevice, c->stream));
    return HX_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free forward pass.  Its work buffers (the packed BF16 input rows
// and the two BF16 hidden layers, [B][ldx] + [B][HID] + [B][HID]) live in one
// file-scope device array per GPU instead of the context's batch buffers,
// which grow with hipMalloc.  The array keeps the last call's contents; every
// entry a call reads is first written by that call (k_pack writes the padding
// columns too), so nothing needs clearing.  Calls that overlap on one GPU
// share the array and race.
constexpr size_t NOALLOC_BYTES = (size_t)16 << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEV = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEV] = {};
}  // namespace

// Device address of this GPU's copy of the array (the array's name in host
// code is only a stand-in).  Called by hx_create with the context's device
// current, once per device.
hx_status noalloc_init(hx_ctx *c)
{
    if (c->device < 0 || c->device >= NOALLOC_MAX_DEV)
        return fail(c, HX_ERR_DEVICE, "device %d beyond the %d supported", c->device, NOALLOC_MAX_DEV);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[c->device]) return HX_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(c, HX_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[c->device] = ptr;
    return HX_OK;
}

int64_t mlp_noalloc_max_batch(const hx_ctx *c)
{
    const int64_t n_in = c->nd + 6 * c->nf + 1, ldx = ((n_in + 31) / 32) * 32;
    return (int64_t)(NOALLOC_BYTES / (size_t)(2 * (ldx + 2 * HID)));
}

hx_status mlp_forward_noalloc(hx_ctx *c, const float *feats, int64_t B, float *out)
{
    if (!c->mlp) return fail(c, HX_ERR_STATE, "no network loaded");
    MlpState *s = c->mlp;
    const int64_t bmax = mlp_noalloc_max_batch(c);
    if (B > bmax)
        return fail(c, HX_ERR_ARG, "batch %lld exceeds the allocation-free maximum %lld (%zu bytes of scratch)",
                    (long long)B, (long long)bmax, NOALLOC_BYTES);
    if (B == 0) return HX_OK;
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = (unsigned char *)g_scratch_ptr[c->device];
    }
    if (!base) return fail(c, HX_ERR_STATE, "scratch of device %d not initialised", c->device);
    uint16_t *xb = (uint16_t *)base;
    uint16_t *h1b = xb + (size_t)B * s->ldx;
    uint16_t *h2b = h1b + (size_t)B * HID;
    hipLaunchKernelGGL(k_pack, dim3(nb256(B * s->ldx)), dim3(256), 0, c->stream, B, s->n_in, s->ldx,
                       feats, xb);
    HX_HIP(c, hipGetLastError());
    HX_HIP(c, gemm(c->stream, (int)B, HID, s->ldx, xb, s->ldx, 1, s->w1b, s->ldx, 1, s->w + s->off_b1,
                   1, nullptr, HID, h1b, HID));
    HX_HIP(c, gemm(c->stream, (int)B, HID, HID, h1b, HID, 1, s->w2b, HID, 1, s->w + s->off_b2, 1,
                   nullptr, HID, h2b, HID));
    HX_HIP(c, gemm(c->stream, (int)B, s->n_out, HID, h2b, HID, 1, s->w3b, HID, 1, s->w + s->off_b3, 0,
                   out, s->n_out, nullptr, 0));
    return HX_OK;
}

hx_status mlp_train(hx_ctx *c, const float *feats, const float *targets, int64_t B, float lr,
                    float *loss_out, float *grad_out)
{
    if (!c->mlp) return fail(c, HX_ERR_STATE, "no network loaded");
    MlpState *s = c->mlp;
    hx_status st = ensure_batch(c, B);
    if (st != HX_OK) return st;
    const hipStream_t q = c->stream;
    hipLaunchKernelGGL(k_pack, dim3(nb256(B * s->ldx)), dim3(256), 0, q, B, s->n_in, s->ldx, feats,
                       s->xb);
    HX_HIP(c, forward_packed(c, B, true));
    const int64_t tot = B * s->n_out;
    const int nbk = (int)std::min<int64_t>(1024, (tot + 255) / 256);
    hipLaunchKernelGGL(k_loss_grad, dim3(nbk), dim3(256), 0, q, tot, 1.0f / (float)tot, s->o, targets,
                       s->d_o, s->dob, s->part);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, q, nbk, s->part, 1.0 / (double)tot, s->loss);
    HX_HIP(c, hipGetLastError());
    float *g = s->grad;
    // layer 3: dW3[o][h] = sum_b dO[b][o] H2[b][h]; db3 = colsum(dO); dH2 = dO W3
    HX_HIP(c, gemm(q, s->n_out, HID, (int)B, s->dob, 1, s->n_out, s->h2b, 1, HID, nullptr, 0,
                   g + s->off_w3, HID, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3(s->n_out), dim3(256), 0, q, B, s->n_out, s->d_o, g + s->off_b3);
    HX_HIP(c, gemm(q, (int)B, HID, s->n_out, s->dob, s->n_out, 1, s->w3b, 1, HID, nullptr, 0, s->dh2,
                   HID, nullptr, 0));
    hipLaunchKernelGGL(k_relu_back, dim3(nb256(B * HID)), dim3(256), 0, q, B * HID, s->h2, s->dh2, s->dh2b);
    // layer 2
    HX_HIP(c, gemm(q, HID, HID, (int)B, s->dh2b, 1, HID, s->h1b, 1, HID, nullptr, 0, g + s->off_w2,
                   HID, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3(HID), dim3(256), 0, q, B, HID, s->dh2, g + s->off_b2);
    HX_HIP(c, gemm(q, (int)B, HID, HID, s->dh2b, HID, 1, s->w2b, 1, HID, nullptr, 0, s->dh1, HID,
                   nullptr, 0));
    hipLaunchKernelGGL(k_relu_back, dim3(nb256(B * HID)), dim3(256), 0, q, B * HID, s->h1, s->dh1, s->dh1b);
    // layer 1: dW1[h][i] = sum_b dH1[b][h] X[b][i] (only the n_in real columns)
    HX_HIP(c, gemm(q, HID, s->n_in, (int)B, s->dh1b, 1, HID, s->xb, 1, s->ldx, nullptr, 0,
                   g + s->off_w1, s->n_in, nullptr, 0));
    hipLaunchKernelGGL(k_colsum, dim3(HID), dim3(256), 0, q, B, HID, s->dh1, g + s->off_b1);
    HX_HIP(c, hipGetLastError());
    s->trace_B = B;
    if (grad_out)
        HX_HIP(c, hipMemcpyAsync(grad_out, g, 4 * (size_t)s->P, hipMemcpyDeviceToDevice, q));
    if (lr != 0.0f) {
        s->t += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)s->t), c2 = 1.f - powf(b2, (float)s->t);
        hipLaunchKernelGGL(k_adam, dim3(nb256(s->P)), dim3(256), 0, q, s->P, s->w, g, s->m, s->v, lr,
                           b1, b2, 1e-8f, c1, c2);
        HX_HIP(c, refresh_bf16(c));
    }
    if (loss_out) {
        HX_HIP(c, hipMemcpyAsync(s->loss_host, s->loss, 4, hipMemcpyDeviceToHost, q));
        HX_HIP(c, hipStreamSynchronize(q));
        *loss_out = s->loss_host[0];
    }
    return HX_OK;
}

hx_status mlp_trace(hx_ctx *c, int what, float *host_buf, int64_t count)
{
    MlpState *s = c->mlp;
    if (!s || s->trace_B == 0) return fail(c, HX_ERR_STATE, "no training step to trace");
    const int64_t B = s->trace_B;
    const float *src = nullptr;
    int width = HID;
    switch (what) {
    case HX_TRACE_INPUT: width = s->n_in; break;
    case HX_TRACE_H1: src = s->h1; break;
    case HX_TRACE_H2: src = s->h2; break;
    case HX_TRACE_OUT: src = s->o; width = s->n_out; break;
    case HX_TRACE_DOUT: src = s->d_o; width = s->n_out; break;
    case HX_TRACE_DH2: src = s->dh2; break;
    case HX_TRACE_DH1: src = s->dh1; break;
    default: return fail(c, HX_ERR_ARG, "unknown trace %d", what);
    }
    if (count != B * width)
        return fail(c, HX_ERR_ARG, "trace %d has %lld values, buffer holds %lld", what,
                    (long long)(B * width), (long long)count);
    if (src) {
        HX_HIP(c, hipMemcpyAsync(host_buf, src, 4 * (size_t)count, hipMemcpyDeviceToHost, c->stream));
        HX_HIP(c, hipStreamSynchronize(c->stream));
        return HX_OK;
    }
    // the packed BF16 inputs: rows of ldx, the first n_in columns widened to FP32
    std::vector<uint16_t> tmp((size_t)B * s->ldx);
    HX_HIP(c, hipMemcpyAsync(tmp.data(), s->xb, 2 * tmp.size(), hipMemcpyDeviceToHost, c->stream));
    HX_HIP(c, hipStreamSynchronize(c->stream));
    for (int64_t b = 0; b < B; ++b)
        for (int j = 0; j < s->n_in; ++j) {
            const uint32_t u = (uint32_t)tmp[(size_t)b * s->ldx + j] << 16;
            std::memcpy(&host_buf[b * s->n_in + j], &u, 4);
        }
    return HX_OK;
}

// one training pair per cell from a solver iterate xj of A x = b with solution xs:
// r = b - A xj, features(r), targets = (xs - xj - BJ(r)) / RMS(BJ(r)) per cell
hx_status mlp_training_pair(hx_ctx *c, const double *b, const double *xs, const double *xj,
                            float clip, float *feats, float *targets)
{
    MlpState *s = c->mlp;
    if (!s) {
        hx_status st = mlp_create(c);
        if (st != HX_OK) return st;
        s = c->mlp;
    }
    if (!s->zt) {
        hx_status st = dalloc(c, (void **)&s->zt, 2 * sizeof(double) * (size_t)c->n_dofs);
        if (st != HX_OK) return st;
    }
    hx_status st = ensure_batch(c, c->n_cells);
    if (st != HX_OK) return st;
    double *r = s->zt, *z = s->zt + c->n_dofs;
    HX_HIP(c, launch_apply64(c, xj, r, b));
    HX_HIP(c, launch_bj64(c, r, z));
    HX_HIP(c, (mlp_features(c, r, feats, s->scale) == HX_OK) ? hipSuccess : hipErrorUnknown);
    hipLaunchKernelGGL(k_targets, dim3((unsigned)c->n_cells), dim3(128), 0, c->stream, c->nd, xs, xj,
                       z, clip, targets);
    HX_HIP(c, hipGetLastError());
    return HX_OK;
}

// z = BJ(v) + w_K net(features(v))_K, w_K = RMS(BJ(v)_K), with v = w / |w|
// (|w|^2 the fixed-order sum of part[0..nbp), v written to vout) or v = w
// (part null).  With at most one workgroup per compute unit the whole
// preconditioner is one launch (the grid is too small for occupancy to
// matter, and the launch it saves does); on larger meshes the block-Jacobi
// kernel (with the normalisation) runs first and the network kernel, at
// half the registers and twice the occupancy, reads its output.
template <int N>
static hipError_t mlp_fused_n(hx_ctx *c, const double *w, const double *part, int nbp,
                              double *vout, double *z)
{
    MlpState *s = c->mlp;
    const int64_t nwg = (c->n_cells + FT - 1) / FT;
    // (degrees 6 and 7 would spill registers in the one-launch form)
    if constexpr (N <= 6) {
        if (nwg <= s->n_cu) {
            hipLaunchKernelGGL((k_mlp_fused<N, true>), dim3((unsigned)nwg), dim3(64 * FW), 0,
                               c->stream, c->n_cells, w, z, c->nbr, c->coef_feat, s->wfr,
                               s->w + s->off_b1, s->w + s->off_b2, s->w + s->off_b3,
                               c->bjS64, c->bjL64, c->bjC64, part, nbp, vout);
            return hipGetLastError();
        }
    }
    hipError_t e = part ? launch_bj64_scaled(c, w, part, nbp, vout, z) : launch_bj64(c, w, z);
    if (e != hipSuccess) return e;
    const double *v = part ? vout : w;
    hipLaunchKernelGGL((k_mlp_fused<N, false>), dim3((unsigned)nwg), dim3(64 * FW), 0, c->stream,
                       c->n_cells, v, z, c->nbr, c->coef_feat, s->wfr,
                       s->w + s->off_b1, s->w + s->off_b2, s->w + s->off_b3, (const double *)nullptr,
                       (const double *)nullptr, (const double *)nullptr, (const double *)nullptr, 0,
                       (double *)nullptr);
    return hipGetLastError();
}

hx_status mlp_apply_fused(hx_ctx *c, const double *w, const double *part, int nbp, double *vout,
                          double *z)
{
    if (!c->mlp) return fail(c, HX_ERR_STATE, "no network loaded");
    hipError_t e = hipSuccess;
    switch (c->n) {
    case 2: e = mlp_fused_n<2>(c, w, part, nbp, vout, z); break;
    case 3: e = mlp_fused_n<3>(c, w, part, nbp, vout, z); break;
    case 4: e = mlp_fused_n<4>(c, w, part, nbp, vout, z); break;
    case 5: e = mlp_fused_n<5>(c, w, part, nbp, vout, z); break;
    case 6: e = mlp_fused_n<6>(c, w, part, nbp, vout, z); break;
    case 7: e = mlp_fused_n<7>(c, w, part, nbp, vout, z); break;
    default: e = mlp_fused_n<8>(c, w, part, nbp, vout, z); break;
    }
    HX_HIP(c, e);
    return HX_OK;
}

// z = BJ(r) + w_K net(features(r))_K in one launch.  A non-finite z shows up
// in the FGMRES Hessenberg column, where the Givens step rejects it and the
// solver switches to block Jacobi.
hx_status mlp_precondition(hx_ctx *c, const double *r, double *z)
{
    return mlp_apply_fused(c, r, nullptr, 0, nullptr, z);
}

// The batched form of the same preconditioner (features, the three layers
// as separate GEMM launches, block Jacobi, correction); kept for comparison.
hx_status mlp_precondition_batched(hx_ctx *c, const double *r, double *z)
{
    if (!c->mlp) return fail(c, HX_ERR_STATE, "no network loaded");
    MlpState *s = c->mlp;
    hx_status st = ensure_batch(c, c->n_cells);
    if (st != HX_OK) return st;
    hipLaunchKernelGGL(k_features, dim3((unsigned)c->n_cells), dim3(128), 0, c->stream, c->n,
                       c->n_cells, r, c->nbr, c->coef_feat, (float *)nullptr, (int64_t)0, s->xb,
                       (int64_t)s->ldx, s->scale);
    HX_HIP(c, hipGetLastError());
    HX_HIP(c, forward_packed(c, c->n_cells, false));
    HX_HIP(c, launch_bj64(c, r, z));
    hipLaunchKernelGGL(k_add_correction, dim3((unsigned)c->n_cells), dim3(128), 0, c->stream, c->nd,
                       s->o, z);
    HX_HIP(c, hipGetLastError());
    return HX_OK;
}

}  // namespace hx
