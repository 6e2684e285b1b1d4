// FP64 reductions shared by the force gather and the binning kernel.
#pragma once

#include "internal.h"

namespace mlmix {

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1)
        v += __shfl_xor(v, d);
    return v;
}

// Sum of nb [3]-partials by one 256-thread block in a fixed order (thread
// stride, wave butterfly, then the four waves pairwise); out[2] (kinetic) is
// converted to eV. Every thread of the block calls it.
__device__ inline void reduce_parts(const double *part, int nb, double *out)
{
    __shared__ double sh[3][4];
    double v[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
        for (int q = 0; q < 3; ++q)
            v[q] += part[b * 3 + q];
    for (int q = 0; q < 3; ++q)
        v[q] = wave_sum_d(v[q]);
    int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 3; ++q)
            sh[q][w] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 0; q < 3; ++q)
            out[q] = (sh[q][0] + sh[q][1]) + (sh[q][2] + sh[q][3]);
        out[2] /= kKappa;
    }
}

}  // namespace mlmix
