// Residual norms without a plan and without allocating: srj_residual_static (include/srj.h).
//
// The reduction scratch (per-block partial sums) lives in a file-scope device array, one
// copy per GPU, whose device address is looked up once per device; the kernels read the
// caller's dense arrays directly and form b = (h_x*h_x) f on the fly.  They follow the
// association and reduction order of the plan-based srj_residual, so both give the same
// bits (r = b - A u in binary64, A = dg I minus the weighted neighbour sum; Sec. 5.1 setting).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "../../include/srj.h"
#include "kernels.h"
#include "reduce.h"

namespace srj {
srj_status report(srj_status s, const std::string& msg);
}

using namespace srj;

namespace {

// Residual blocks (up to kResRowsMax lines each) the scratch holds: 2 (sum, max) pairs per block, one
// for r and one for b~ (the residual of the zero interior).  65536 blocks = 524288 lines
// (rows in 2D, (k, i) lines in 3D), 2 MiB.
constexpr int kStaticBlocks = 65536;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[4 * kStaticBlocks];

double* g_scratch[kMaxDevices] = {nullptr};
std::mutex g_scratch_mu;

// Device address of this GPU's scratch array (looked up on the first call per device).
srj_status scratch_ptr(double** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return report(SRJ_EHIP, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return report(SRJ_EINVAL, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return report(SRJ_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return SRJ_OK;
}

__device__ __forceinline__ double ldz_d(const double* u, int64_t p, bool zero) { return zero ? 0.0 : u[p]; }

struct Wts {
    double wy, wz, dg;
};

// r at interior point p of the dense layout (pitch nx + 2, ny + 2 rows per plane), with b
// = hh * f[p] and the operator weights w; zi reads u's interior as 0 (the residual of the
// zero interior is b~).
__device__ __forceinline__ double res_dense(const double* u, const double* f, double hh, const Wts& w, int64_t p,
                                            int64_t px, int64_t pl, int ndim, int i, int j, int k, int nx, int ny,
                                            int nz, bool zi)
{
    const bool zl = zi && j - 1 >= 1, zr = zi && j + 1 <= nx;
    const bool zs = zi && i - 1 >= 1, zn = zi && i + 1 <= ny;
    double s = (ldz_d(u, p - 1, zl) + ldz_d(u, p + 1, zr)) + w.wy * (ldz_d(u, p - px, zs) + ldz_d(u, p + px, zn));
    if (ndim == 3) {
        const bool zd = zi && k - 1 >= 1, zu = zi && k + 1 <= nz;
        s = s + w.wz * (ldz_d(u, p - pl, zd) + ldz_d(u, p + pl, zu));
    }
    return (s + hh * f[p]) - w.dg * ldz_d(u, p, zi);
}

// One block per res_rows(lines) lines: (sum r^2, max |r|) into part[0..2nb) and (sum b~^2, max |b~|)
// into part[2nb..4nb); r_out (may be null) receives r on the interior.
__global__ __launch_bounds__(256) void k_residual_static(const double* __restrict__ u, const double* __restrict__ f,
                                                         double hh, Wts w, int ndim, int nx, int ny, int nz,
                                                         double* __restrict__ r_out, double* __restrict__ part,
                                                         int nb)
{
    const int64_t px = nx + 2, py = ny + 2, pl = px * py;
    const int64_t lines = (int64_t)ny * (ndim == 3 ? nz : 1);
    double s1 = 0.0, m1 = 0.0, s0 = 0.0, m0 = 0.0;
    const int rpb = res_rows(lines);
    const int64_t q0 = (int64_t)blockIdx.x * rpb;
    for (int64_t q = q0; q < min(q0 + rpb, lines); ++q) {
        const int i = (int)(q % ny) + 1;
        const int k = (ndim == 3) ? (int)(q / ny) + 1 : 0;
        const int64_t rowp = (int64_t)k * pl + (int64_t)i * px;
        for (int j = threadIdx.x + 1; j <= nx; j += 256) {
            const double r = res_dense(u, f, hh, w, rowp + j, px, pl, ndim, i, j, k, nx, ny, nz, false);
            const double b = res_dense(u, f, hh, w, rowp + j, px, pl, ndim, i, j, k, nx, ny, nz, true);
            if (r_out) r_out[rowp + j] = r;
            s1 = s1 + r * r;
            nanmax(m1, fabs(r));
            s0 = s0 + b * b;
            nanmax(m0, fabs(b));
        }
    }
    block_reduce(s1, m1);
    __syncthreads();
    block_reduce(s0, m0);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1;
        part[2 * blockIdx.x + 1] = m1;
        part[2 * (int64_t)nb + 2 * blockIdx.x] = s0;
        part[2 * (int64_t)nb + 2 * blockIdx.x + 1] = m0;
    }
}

// Fold the partials in the order of the plan-based reduction and write the four norms.
__global__ __launch_bounds__(256) void k_residual_static_final(const double* __restrict__ part, int nb,
                                                               double* __restrict__ norms)
{
    double s1 = 0.0, m1 = 0.0, s0 = 0.0, m0 = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) {
        s1 = s1 + part[2 * i];
        nanmax(m1, part[2 * i + 1]);
        s0 = s0 + part[2 * nb + 2 * i];
        nanmax(m0, part[2 * nb + 2 * i + 1]);
    }
    block_reduce(s1, m1);
    __syncthreads();
    block_reduce(s0, m0);
    if (threadIdx.x == 0) {
        const double l2 = sqrt(s1), b2 = sqrt(s0);
        norms[0] = l2;
        norms[1] = m1;
        norms[2] = b2;
        norms[3] = s0 > 0.0 ? l2 / b2 : 0.0;
    }
}

// Zero on every ring cell of the dense layout (a fill kernel: nothing here records a memset).
__global__ __launch_bounds__(256) void k_ring_zero(double* __restrict__ r, int ndim, int nx, int ny, int nz)
{
    const int64_t nxw = nx + 2, nyw = ny + 2, nzw = ndim == 3 ? nz + 2 : 1;
    const int64_t n = nxw * nyw * nzw;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx % nxw, t = idx / nxw, i = t % nyw, k = t / nyw;
        const bool ring = j == 0 || j == nx + 1 || i == 0 || i == ny + 1 || (ndim == 3 && (k == 0 || k == nz + 1));
        if (ring) r[idx] = 0.0;
    }
}

}  // namespace

extern "C" srj_status srj_residual_static(const srj_grid* grid, const double* u, const double* f, double* r_out,
                                          double* norms, void* stream)
{
    if (!grid || !u || !f || !norms) return report(SRJ_EINVAL, "null argument");
    if (grid->ndim != 2 && grid->ndim != 3) return report(SRJ_EINVAL, "ndim must be 2 or 3");
    if (grid->bc != 0) return report(SRJ_EINVAL, "Dirichlet grids only");
    for (int i = 0; i < grid->ndim; ++i) {
        if (grid->n[i] < 1 || grid->n[i] > (1 << 20)) return report(SRJ_EINVAL, "n must be in [1, 2^20]");
        if (!(grid->h[i] > 0) || !std::isfinite(grid->h[i])) return report(SRJ_EINVAL, "every h[i] must be positive");
    }
    const int64_t nz = grid->ndim == 3 ? grid->n[2] : 1;
    const int64_t lines = grid->n[1] * nz;
    const int rpb = res_rows(lines);
    const int64_t nb = (lines + rpb - 1) / rpb;
    if (nb > kStaticBlocks)
        return report(SRJ_EINVAL, "grid too large for the static scratch: at most " +
                                      std::to_string((int64_t)kStaticBlocks * kResRowsMax) +
                                      " lines (rows in 2D, n_y * n_z in 3D), got " + std::to_string(lines));
    double* part = nullptr;
    srj_status st = scratch_ptr(&part);
    if (st != SRJ_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Geo g{};
    g.ndim = grid->ndim;
    geo_set_weights(g, grid->h, nullptr);
    const Wts w{g.wy, g.wz, g.dg};
    const double hh = grid->h[0] * grid->h[0];
    const int nx = (int)grid->n[0], ny = (int)grid->n[1];
    if (r_out) {
        const int64_t total = (int64_t)(nx + 2) * (ny + 2) * (grid->ndim == 3 ? nz + 2 : 1);
        const int64_t blocks = std::min<int64_t>(65536, std::max<int64_t>(1, (total + 255) / 256));
        hipLaunchKernelGGL(k_ring_zero, dim3((unsigned)blocks), dim3(256), 0, s, r_out, grid->ndim, nx, ny, (int)nz);
    }
    hipLaunchKernelGGL(k_residual_static, dim3((unsigned)nb), dim3(256), 0, s, u, f, hh, w, grid->ndim, nx, ny, (int)nz,
                       r_out, part, (int)nb);
    hipLaunchKernelGGL(k_residual_static_final, dim3(1), dim3(256), 0, s, (const double*)part, (int)nb, norms);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return report(SRJ_EHIP, std::string("residual launch: ") + hipGetErrorString(e));
    return SRJ_OK;
}
