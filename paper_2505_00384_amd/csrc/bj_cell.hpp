// The cell solve of the separable block Jacobi, shared by the block-Jacobi
// kernels and the learned preconditioner's fused kernel:
//   z_K = (S_z (x) S_y (x) S_x) diag(1/(c0 + cx lx_i + cy ly_j + cz lz_l))
//         (S_z (x) S_y (x) S_x)^T r_K
// (the tensor-product inverse of paper section 3.3 applied to the separable
// approximation of the Helmholtz cell block).
#pragma once

#include <hip/hip_runtime.h>

namespace hx {

// One cell's solve in place in LDS.  sR: the cell's N^3 values (r on entry,
// z on return), x fastest; sS: [3][N*N] per-direction eigenvector matrices
// (sS[d][i*N + m] = S_d(i, m)); sL: [3][N] eigenvalues; sC: c0, cx, cy, cz.
// Thread (a, b) of the cell (a, b < N) owns one pencil per sweep; every
// thread of the workgroup calls this (barriers inside), with active false
// for threads without a cell.  acc_rz accumulates r.z over the thread's
// final pencil (positions i + N a + N^2 b).
template <int N, typename T>
__device__ __forceinline__ void bj_cell_solve(T *sR, const T (*sS)[N * N], const T (*sL)[N],
                                              const T *sC, int a, int b, bool active,
                                              double &acc_rz)
{
    constexpr int NF = N * N;
    T v[N], w[N], rp[N];
    // S_x^T along x: thread (j=a, l=b); rp keeps the residual pencil, whose
    // positions are those of the output pencil written at the end
    if (active) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = rp[i] = sR[i + N * a + NF * b];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            T s = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) s += sS[0][i * N + m] * v[i];
            w[m] = s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int m = 0; m < N; ++m) sR[m + N * a + NF * b] = w[m];
    }
    __syncthreads();
    // S_y^T along y: thread (mx=a, l=b)
    if (active) {
#pragma unroll
        for (int j = 0; j < N; ++j) v[j] = sR[a + N * j + NF * b];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            T s = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) s += sS[1][j * N + m] * v[j];
            w[m] = s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int m = 0; m < N; ++m) sR[a + N * m + NF * b] = w[m];
    }
    __syncthreads();
    // S_z^T along z, diagonal scaling, S_z along z: thread (mx=a, my=b)
    if (active) {
#pragma unroll
        for (int l = 0; l < N; ++l) v[l] = sR[a + N * b + NF * l];
        const T c0 = sC[0], cx = sC[1], cy = sC[2], cz = sC[3];
        const T base = c0 + cx * sL[0][a] + cy * sL[1][b];
#pragma unroll
        for (int m = 0; m < N; ++m) {
            T s = 0;
#pragma unroll
            for (int l = 0; l < N; ++l) s += sS[2][l * N + m] * v[l];
            w[m] = s / (base + cz * sL[2][m]);
        }
#pragma unroll
        for (int l = 0; l < N; ++l) {
            T s = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) s += sS[2][l * N + m] * w[m];
            v[l] = s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int l = 0; l < N; ++l) sR[a + N * b + NF * l] = v[l];
    }
    __syncthreads();
    // S_y along y: thread (mx=a, l=b)
    if (active) {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = sR[a + N * m + NF * b];
#pragma unroll
        for (int j = 0; j < N; ++j) {
            T s = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) s += sS[1][j * N + m] * v[m];
            w[j] = s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int j = 0; j < N; ++j) sR[a + N * j + NF * b] = w[j];
    }
    __syncthreads();
    // S_x along x: thread (j=a, l=b); the result goes back through LDS so
    // that the callers' stores are contiguous across threads
    if (active) {
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = sR[m + N * a + NF * b];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            T s = 0;
#pragma unroll
            for (int m = 0; m < N; ++m) s += sS[0][i * N + m] * v[m];
            w[i] = s;
            acc_rz += (double)rp[i] * (double)s;
        }
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < N; ++i) sR[i + N * a + NF * b] = w[i];
    }
    __syncthreads();
}

}  // namespace hx
