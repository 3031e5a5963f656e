// A whole SRJ solve of a small 2D grid in one workgroup, the grid resident in LDS.
//
// For grids whose iterate pair and source fit in the compute unit's LDS (binary64, at most
// kSmallPoints points with the ring: 64 x 64 interior is 4356) one launch runs every sweep,
// the residual checks at cycle ends (Sec. 2's M-cycles; the stopping rule of srj_solve) and
// the final write-back; the host synchronises once.  Launch and check overheads dominate
// such grids otherwise: a 64^2 solve needs about 5000 sweeps of 4096 points each.
//
// The arithmetic per point is the sweep of the other kernels (Sec. 3.1, Eq. 2nd-order_CD):
//     s = (W + E) + wy (S + N);  t = (s + b) - dg u;  u' = u + c t
// in that association with every operation rounded on its own, so the iterates are the
// oracle's bit for bit.  The residual norms are binary64 sums in the workgroup's own order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "kernels.h"

namespace srj {

namespace {

constexpr int kSmallThreads = 1024;

// Sum and max over the workgroup: a shuffle-xor butterfly in each wave, then the 16 wave
// results in order by thread 0; every thread returns the totals.
__device__ __forceinline__ void small_reduce(double& s, double& m, double* red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double so = __shfl_xor(s, o, 64);
        const double mo = __shfl_xor(m, o, 64);
        s = s + so;
        if (mo > m || mo != mo) m = mo;
    }
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[2 * w] = s;
        red[2 * w + 1] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ts = 0.0, tm = 0.0;
        for (int i = 0; i < kSmallThreads / 64; ++i) {
            ts = ts + red[2 * i];
            if (red[2 * i + 1] > tm || red[2 * i + 1] != red[2 * i + 1]) tm = red[2 * i + 1];
        }
        red[2 * (kSmallThreads / 64)] = ts;
        red[2 * (kSmallThreads / 64) + 1] = tm;
    }
    __syncthreads();
    s = red[2 * (kSmallThreads / 64)];
    m = red[2 * (kSmallThreads / 64) + 1];
}

// in: field (padded, pitch px) with the start and its ring; b: padded source; cseq[M]: the
// cycle's coefficients; out: the returned state (padded); res = {sweeps, cycles, relres,
// status} (status as srj_status: OK, ENOCONV, EDIVERGED).
__global__ __launch_bounds__(kSmallThreads) void k_small_solve(const double* __restrict__ in,
                                                               const double* __restrict__ bsrc,
                                                               double* __restrict__ out, Geo g,
                                                               const double* __restrict__ cseq, int64_t M,
                                                               double tol, int64_t max_sweeps,
                                                               double* __restrict__ res)
{
    __shared__ double lds[3 * kSmallPoints];
    __shared__ double red[2 * (kSmallThreads / 64) + 2];
    const int nx = (int)g.nx, ny = (int)g.ny, w = nx + 2;
    const int npts = w * (ny + 2);
    double* ua = lds;
    double* ub = lds + npts;
    double* bl = lds + 2 * npts;
    for (int idx = threadIdx.x; idx < npts; idx += kSmallThreads) {
        const int i = idx / w, j = idx % w;
        const double v = in[(int64_t)i * g.px + j];
        ua[idx] = v;
        ub[idx] = v;
        bl[idx] = bsrc[(int64_t)i * g.px + j];
    }
    __syncthreads();
    const int n = nx * ny;
    const double wy = g.wy, dg = g.dg;
    // residual norms of state u (zero: read the interior as 0)
    auto residual = [&](const double* u, bool zero, double* sum) {
        double s = 0.0, m = 0.0;
        for (int idx = threadIdx.x; idx < n; idx += kSmallThreads) {
            const int i = idx / nx + 1, j = idx % nx + 1;
            const int p = i * w + j;
            const bool il = j > 1, ir = j < nx, is = i > 1, in_ = i < ny;
            const double W = (zero && il) ? 0.0 : u[p - 1], E = (zero && ir) ? 0.0 : u[p + 1];
            const double S = (zero && is) ? 0.0 : u[p - w], N = (zero && in_) ? 0.0 : u[p + w];
            const double sm = (W + E) + wy * (S + N);
            const double r = (sm + bl[p]) - dg * (zero ? 0.0 : u[p]);
            s = s + r * r;
            const double a = fabs(r);
            if (a > m || a != a) m = a;
        }
        small_reduce(s, m, red);
        *sum = s;
    };
    double bt2;
    residual(ua, true, &bt2);
    double* cur = ua;
    double* nxt = ub;
    int64_t k = 0, cycles = 0;
    double rr = 0.0;
    int status = 0;
    if (!isfinite(bt2)) {
        status = 6;
        rr = NAN;
    } else if (bt2 == 0.0) {
        for (int idx = threadIdx.x; idx < n; idx += kSmallThreads) cur[(idx / nx + 1) * w + idx % nx + 1] = 0.0;
        __syncthreads();
    } else {
        for (;;) {
            double r2;
            residual(cur, false, &r2);
            rr = sqrt(r2) / sqrt(bt2);
            if (!isfinite(rr)) {
                status = 6;
                break;
            }
            if (rr <= tol) break;
            if (k + M > max_sweeps) {
                status = 5;
                break;
            }
            for (int64_t s = 0; s < M; ++s) {
                const double c = cseq[s];
                for (int idx = threadIdx.x; idx < n; idx += kSmallThreads) {
                    const int p = (idx / nx + 1) * w + idx % nx + 1;
                    const double m = cur[p];
                    const double sm = (cur[p - 1] + cur[p + 1]) + wy * (cur[p - w] + cur[p + w]);
                    const double t = (sm + bl[p]) - dg * m;
                    nxt[p] = m + c * t;
                }
                __syncthreads();
                double* tmp = cur;
                cur = nxt;
                nxt = tmp;
            }
            k += M;
            cycles += 1;
        }
    }
    for (int idx = threadIdx.x; idx < npts; idx += kSmallThreads) {
        const int i = idx / w, j = idx % w;
        out[(int64_t)i * g.px + j] = cur[idx];
    }
    if (threadIdx.x == 0) {
        res[0] = (double)k;
        res[1] = (double)cycles;
        res[2] = rr;
        res[3] = (double)status;
    }
}

}  // namespace

bool small_solve_fits(const Geo& g)
{
    return g.ndim == 2 && g.bc == 0 && !g.op && (g.nx + 2) * (g.ny + 2) <= kSmallPoints;
}

hipError_t launch_small_solve(const double* in, const double* b, double* out, const Geo& g, const double* cseq,
                              int64_t M, double tol, int64_t max_sweeps, double* res, hipStream_t s)
{
    if (!small_solve_fits(g)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_small_solve, dim3(1), dim3(kSmallThreads), 0, s, in, b, out, g, cseq, M, tol, max_sweeps,
                       res);
    return hipGetLastError();
}

}  // namespace srj
