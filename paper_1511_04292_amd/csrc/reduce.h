// Block reductions of the residual kernels: (sum, max) pairs over 256-thread blocks, in a
// fixed order so that every launch with the same data gives the same bits.
#pragma once

#include <hip/hip_runtime.h>

namespace srj {

// Lines (rows in 2D, (k, i) lines in 3D) per residual block: as many blocks as fill the
// device (about kResBlocks) while a block takes at most kResRowsMax lines, so that large
// grids leave few partial sums.  Every kernel that reduces a residual uses this geometry,
// which fixes the order of its sums.
constexpr int kResRowsMax = 8;
constexpr int64_t kResBlocks = 1024;
__host__ __device__ inline int res_rows(int64_t lines)
{
    const int64_t r = lines / kResBlocks;
    return (int)(r < 1 ? 1 : (r > kResRowsMax ? kResRowsMax : r));
}

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
