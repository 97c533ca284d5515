// Fixed-order workgroup sum shared by the kernels that reduce the same
// partial sums independently (every workgroup of a launch, or two different
// kernels, obtain the same bits).
#pragma once

#include <hip/hip_runtime.h>

namespace hx {

// Sum of p[0..nb) by the first 256 threads of a workgroup of at least 256
// (every thread calls it): thread t < 256 adds p[t], p[t + 256], ...
// starting from 0; each wave folds its lanes with shuffle-down distances 32,
// 16, ..., 1; the four wave sums are added in wave order starting from 0.
// Every thread returns the result.  The host function host_sum256
// (solver.cpp) performs the same additions in the same order.
__device__ inline double sum256(const double *__restrict__ p, int nb, double *sh /* LDS [4] */)
{
    double s = 0.0;
    if (threadIdx.x < 256)
        for (int i = threadIdx.x; i < nb; i += 256) s += p[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0 && wv < 4) sh[wv] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) t += sh[q];
    __syncthreads();
    return t;
}

}  // namespace hx
