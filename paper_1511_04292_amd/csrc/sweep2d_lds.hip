// Temporally blocked 2D sweeps with the tile held in LDS, for the binary64 operators that the
// register-streamed kernel does not cover: unequal spacings, homogeneous Neumann boundaries
// (Sec. 3.1's model problem) and operators given point by point with a mask (Sec. 5.3).
//
// One workgroup of 1024 threads owns an output tile of O x O points (O = 32 or 64, below).  It loads the tile with an
// 8-point halo (O + 16 points square of u, b and, for operators, the four scaled neighbour
// weights and the mask) into LDS once, applies up to 8 scheduled sweeps there -- level l
// updates the window less l points on each side, whose neighbours the previous level has
// updated -- and writes the tile's own points back.  Neighbouring tiles recompute each other's halos.  Each sweep is the
// one-sweep kernels' arithmetic point for point:
//     Poisson   s = (W + E) + wy (S + N);  t = (s + b) - dg u;  u' = u + c t
//     operator  s = (wW W + wE E) + (wS S + wN N);  t = (s + b) - u;  u' = u + c t
// every operation rounded on its own, so the iterates are those of T unfused sweeps bit for
// bit.  With Neumann boundaries a neighbour across the boundary is the point itself; ring
// points (Dirichlet data) and masked points keep their values.
//
// On small grids (up to about a million points) the one-sweep kernels are bound by launch
// latency; here a launch does T sweeps out of LDS for one pass over HBM.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace srj {

namespace {

enum { LDS_POISSON = 0, LDS_NEUMANN = 1, LDS_OPERATOR = 2 };

constexpr int kLdsThreads = 1024;
constexpr int kLdsT = 8;  // largest number of sweeps per launch

// Output tiles are O x O points.  Poisson (Dirichlet or Neumann) loads u twice and b: at O = 64
// an 80 x 80 window, 150 KiB of LDS, for large grids; at O = 32 a 48 x 48 window, 54 KiB (two
// workgroups per compute unit), for grids that would give fewer than kLdsBigTiles large tiles,
// where a launch's latency (the points each thread walks per level) is what counts.
// Operators (O = 32) also load four weights and the mask: 128 KiB.
constexpr int kLdsBigTiles = 512;

template <int MODE, int O> struct LdsExtra {
    __device__ void load(int, int64_t, const Geo&) {}
};
template <int O> struct LdsExtra<LDS_OPERATOR, O> {
    static constexpr int L = O + 2 * kLdsT;
    double w[4][L * L];
    uint8_t mask[L * L];
    __device__ void load(int idx, int64_t p, const Geo& g)
    {
#pragma unroll
        for (int k = 0; k < 4; ++k) w[k][idx] = g.w[k][p];
        mask[idx] = g.mask ? g.mask[p] : (uint8_t)0;
    }
};

template <int MODE, int O>
__global__ __launch_bounds__(kLdsThreads) void k_sweep2d_lds(const double* __restrict__ in, double* __restrict__ out,
                                                             const double* __restrict__ bsrc, Geo g, Coefs co,
                                                             int Tact, int ntx)
{
    constexpr int L = O + 2 * kLdsT;  // loaded window, square
    __shared__ double su[2][L * L];
    __shared__ double sb[L * L];
    __shared__ LdsExtra<MODE, O> ex;

    const int nx = (int)g.nx, ny = (int)g.ny;
    const int tx = (int)blockIdx.x % ntx, ty = (int)blockIdx.x / ntx;
    // grid coordinates of window point (0, 0); the window is centred on the tile whatever T is
    const int x0 = 1 + tx * O - kLdsT, y0 = 1 + ty * O - kLdsT;

    for (int idx = threadIdx.x; idx < L * L; idx += kLdsThreads) {
        const int ly = idx / L, lx = idx % L;
        const int gy = min(max(y0 + ly, 0), ny + 1), gx = min(max(x0 + lx, 0), nx + 1);
        const int64_t p = (int64_t)gy * g.px + gx;
        const double v = in[p];
        su[0][idx] = v;
        su[1][idx] = v;
        sb[idx] = bsrc[p];
        ex.load(idx, p, g);
    }
    __syncthreads();

    const double wy = g.wy, dg = g.dg;
    int cur = 0;
    for (int l = 1; l <= Tact; ++l) {
        const double c = co.c[l - 1];
        // level l updates the band [l, L - l) of the window on both axes: the neighbours it
        // reads lie in the band of level l - 1; after Tact <= kLdsT levels the band still
        // holds the tile's own points [kLdsT, kLdsT + O)
        const double* __restrict__ a = su[cur];
        double* __restrict__ z = su[cur ^ 1];
        for (int idx = threadIdx.x; idx < L * L; idx += kLdsThreads) {
            const int ly = idx / L, lx = idx % L;
            if (ly < l || ly >= L - l || lx < l || lx >= L - l) continue;
            const int gy = y0 + ly, gx = x0 + lx;
            if (gy < 1 || gy > ny || gx < 1 || gx > nx) continue;  // ring and beyond: fixed
            const double m = a[idx];
            if constexpr (MODE == LDS_OPERATOR) {
                if (ex.mask[idx]) {
                    z[idx] = m;
                    continue;
                }
                const double s = (ex.w[0][idx] * a[idx - 1] + ex.w[1][idx] * a[idx + 1]) +
                                 (ex.w[2][idx] * a[idx - L] + ex.w[3][idx] * a[idx + L]);
                const double t = (s + sb[idx]) - m;
                z[idx] = m + c * t;
            } else {
                const bool neu = MODE == LDS_NEUMANN;
                const double W = (neu && gx == 1) ? m : a[idx - 1];
                const double E = (neu && gx == nx) ? m : a[idx + 1];
                const double S = (neu && gy == 1) ? m : a[idx - L];
                const double N = (neu && gy == ny) ? m : a[idx + L];
                const double s = (W + E) + wy * (S + N);
                const double t = (s + sb[idx]) - dg * m;
                z[idx] = m + c * t;
            }
        }
        __syncthreads();
        cur ^= 1;
    }

    for (int idx = threadIdx.x; idx < O * O; idx += kLdsThreads) {
        const int oy = idx / O, ox = idx % O;
        const int gy = 1 + ty * O + oy, gx = 1 + tx * O + ox;
        if (gy > ny || gx > nx) continue;
        out[(int64_t)gy * g.px + gx] = su[cur][(oy + kLdsT) * L + ox + kLdsT];
    }
}

template <int MODE, int O>
hipError_t lds_launch(const double* in, double* out, const double* b, const Geo& g, const Coefs& co, int T,
                      hipStream_t s)
{
    const int ntx = (int)((g.nx + O - 1) / O), nty = (int)((g.ny + O - 1) / O);
    hipLaunchKernelGGL((k_sweep2d_lds<MODE, O>), dim3((unsigned)(ntx * nty)), dim3(kLdsThreads), 0, s, in, out, b, g,
                       co, T, ntx);
    return hipGetLastError();
}

template <int MODE>
hipError_t lds_launch_poisson(const double* in, double* out, const double* b, const Geo& g, const Coefs& co, int T,
                              hipStream_t s)
{
    const int64_t big = ((g.nx + 63) / 64) * ((g.ny + 63) / 64);
    if (big >= kLdsBigTiles) return lds_launch<MODE, 64>(in, out, b, g, co, T, s);
    return lds_launch<MODE, 32>(in, out, b, g, co, T, s);
}

}  // namespace

int lds_fuse_max() { return kLdsT; }

bool lds_fuse_fits(const Geo& g, Fmt f)
{
    // 2D binary64, tile counts within a launch grid
    return g.ndim == 2 && f == FMT_F64 && g.nx <= (1 << 20) && g.ny <= (1 << 20) &&
           ((g.nx + 31) / 32) * ((g.ny + 31) / 32) < ((int64_t)1 << 31);
}

hipError_t launch_sweep_lds2d(const void* in, void* out, const void* b, const Geo& g, const Coefs& co, int T,
                              hipStream_t s)
{
    if (g.ndim != 2 || T < 1 || T > kLdsT) return hipErrorInvalidValue;
    const double* i = (const double*)in;
    double* o = (double*)out;
    const double* bb = (const double*)b;
    if (g.op) return lds_launch<LDS_OPERATOR, 32>(i, o, bb, g, co, T, s);
    if (g.bc == 1) return lds_launch_poisson<LDS_NEUMANN>(i, o, bb, g, co, T, s);
    return lds_launch_poisson<LDS_POISSON>(i, o, bb, g, co, T, s);
}

}  // namespace srj
