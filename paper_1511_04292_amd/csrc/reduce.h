// Block reductions of the residual kernels: (sum, max) pairs over 256-thread blocks, in a
// fixed order so that every launch with the same data gives the same bits.
#pragma once

#include <hip/hip_runtime.h>

namespace srj {

constexpr int kResRows = 8;  // rows (2D) or (k, i) lines (3D) per residual block

// max that keeps a NaN once one is seen
__device__ __forceinline__ void nanmax(double& m, double a)
{
    if (a > m || a != a) m = a;
}

// Block reduction of (sum, max) over 256 threads: a shuffle-xor butterfly inside each wave,
// then the 4 wave results in a fixed order.  Thread 0 returns the result.  Calls that follow
// one another in a kernel must be separated by a barrier (they share the LDS slots).
__device__ __forceinline__ void block_reduce(double& s, double& m)
{
    __shared__ double ss[4], sm[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double so = __shfl_xor(s, o, 64);
        double mo = __shfl_xor(m, o, 64);
        s = s + so;
        nanmax(m, mo);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ss[w] = s;
        sm[w] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s = (ss[0] + ss[1]) + (ss[2] + ss[3]);
        m = sm[0];
        nanmax(m, sm[1]);
        nanmax(m, sm[2]);
        nanmax(m, sm[3]);
    }
}

}  // namespace srj
