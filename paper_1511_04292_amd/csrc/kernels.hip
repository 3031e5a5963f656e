// SRJ device kernels for gfx950 (CDNA4, wave64).
//
// The weighted-Jacobi step (Sec. 3.1, Eq. 2nd-order_CD, Poisson form with b = h_x^2 f):
//     s = (W + E) + wy (S + N)  [ + wz (D + U) in 3D ]
//     t = (s + b) - dg * u
//     u' = u + c * t,        c = w / dg
// with exactly this association and no fused multiply-add (the file is built with
// -ffp-contract=off), so every kernel below -- unfused or temporally blocked -- produces
// bit-identical iterates for the same sweep sequence.  wy, wz and dg are the weights of a
// box whose axes have different spacings (Geo); with equal spacings they are 1, 1 and 2d,
// every product by them is exact, and the register-streamed temporally blocked kernels,
// which implement that case only, give the same bits.  Storage formats: binary64,
// binary32, and bfloat16 (binary32 arithmetic, round-to-nearest-even on every store).
//
// The sweep is bound by HBM bandwidth (0.3 flop per byte unfused), so no kernel uses the
// matrix cores.  This file holds the one-sweep kernels (with the sweep that also forms the
// residual of its input), data movement, residual reductions, operator set-up and refinement
// helpers.  Elsewhere: the temporally blocked sweeps (sweep2d_tb.hip, sweep3d_tb.hip, and
// sweep2d_lds.hip for unequal spacings, Neumann boundaries and operators), the whole small
// solve in LDS (small_solve.hip), the batch (batch.hip) and the allocation-free residual
// (residual_static.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "formats.h"
#include "tb_core.h"
#include "kernels.h"
#include "reduce.h"

namespace srj {

size_t fmt_size(Fmt f) { return f == FMT_F64 ? 8 : (f == FMT_F32 ? 4 : 2); }

// ------------------------------------------------------------ copy / rhs / fill

template <class S>
__global__ __launch_bounds__(256) void k_copy_in(const double* __restrict__ user, S* __restrict__ f,
                                                 Geo g)
{
    const int64_t rows = (g.ndim == 3 ? g.nz + 2 : 1) * g.py;
    const int64_t w = g.nx + 2;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < rows * w;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t row = idx / w, j = idx % w;
        f[row * g.px + j] = Tr<S>::from64(user[idx]);
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_copy_out(const S* __restrict__ f, double* __restrict__ user,
                                                  Geo g)
{
    const int64_t planes = (g.ndim == 3 ? g.nz : 1);
    const int64_t n = planes * g.ny * g.nx;
    const int64_t w = g.nx + 2;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = idx % g.nx + 1;
        int64_t t = idx / g.nx;
        int64_t i = t % g.ny + 1;
        int64_t k = (g.ndim == 3) ? t / g.ny + 1 : 0;
        int64_t row = k * g.py + i;
        user[row * w + j] = (double)Tr<S>::ld(f[row * g.px + j]);
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_rhs(const double* __restrict__ uf, double hh, S* __restrict__ blo,
                                             double* __restrict__ b64, Geo g)
{
    const int64_t planes = (g.ndim == 3 ? g.nz : 1);
    const int64_t n = planes * g.ny * g.nx;
    const int64_t w = g.nx + 2;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = idx % g.nx + 1;
        int64_t t = idx / g.nx;
        int64_t i = t % g.ny + 1;
        int64_t k = (g.ndim == 3) ? t / g.ny + 1 : 0;
        int64_t row = k * g.py + i;
        double b = hh * uf[row * w + j];
        if (b64) b64[row * g.px + j] = b;
        if (blo) blo[row * g.px + j] = Tr<S>::from64(b);
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_zero(S* __restrict__ f, int64_t n)
{
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x)
        f[idx] = zero_of<S>();
}

// ------------------------------------------------------------- unfused sweeps

// One sweep, one thread per interior point (reference kernel; also small grids).
// NEU: homogeneous Neumann boundaries (Sec. 3.1 model problem): a neighbour across the
// boundary is the cell itself.
template <class S, bool NEU>
__global__ __launch_bounds__(256) void k_sweep2d(const S* __restrict__ u, S* __restrict__ o,
                                                 const S* __restrict__ b, int64_t px, int nx, int ny,
                                                 double wy64, double dg64, double c64)
{
    using Cm = typename Tr<S>::C;
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i = blockIdx.y * 4 + threadIdx.y + 1;
    if (j > nx || i > ny) return;
    const Cm c = (Cm)c64, wy = (Cm)wy64, dg = (Cm)dg64;
    const int64_t p = (int64_t)i * px + j;
    const int64_t pw = (NEU && j == 1) ? p : p - 1, pe = (NEU && j == nx) ? p : p + 1;
    const int64_t ps = (NEU && i == 1) ? p : p - px, pn = (NEU && i == ny) ? p : p + px;
    Cm m = Tr<S>::ld(u[p]);
    Cm s = (Tr<S>::ld(u[pw]) + Tr<S>::ld(u[pe])) + wy * (Tr<S>::ld(u[ps]) + Tr<S>::ld(u[pn]));
    Cm t = (s + Tr<S>::ld(b[p])) - dg * m;
    o[p] = Tr<S>::st(m + c * t);
}

// One 3D sweep: threads over (x, y) (block of 64 x BY), each walking a run of z planes with
// the z neighbours and D planes ahead kept in registers.  The y neighbours of a block's rows
// come from its own loads through L1 except on its first and last row, so taller blocks
// fetch fewer extra rows from HBM.  The z loop is branch-free (clamped plane index; the
// stores of planes past the run are dropped by the range check of a buffer resource that
// covers the run) so the loads of the next D planes stay in flight while a plane computes.
template <class S, int D, bool NEU>
__global__ __launch_bounds__(1024) void k_sweep3d(const S* __restrict__ u, S* __restrict__ o,
                                                  const S* __restrict__ b, int64_t px, int64_t py,
                                                  int nx, int ny, int nz, int zrun, double wy64, double wz64,
                                                  double dg64, double c64)
{
    using Cm = typename Tr<S>::C;
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i = blockIdx.y * blockDim.y + threadIdx.y + 1;
    if (j > nx || i > ny) return;
    const int k0 = blockIdx.z * zrun + 1;
    const int k1 = min(k0 + zrun, nz + 1);
    const Cm c = (Cm)c64, wy = (Cm)wy64, wz = (Cm)wz64, dg = (Cm)dg64;
    const int64_t pl = px * py;
    const int64_t col = (int64_t)i * px + j;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(o + (int64_t)k0 * pl), (short)0, (int)((int64_t)(k1 - k0) * pl * (int64_t)sizeof(S)), 0x00020000);
    Cm dn = Tr<S>::ld(u[(int64_t)(k0 - 1) * pl + col]);
    Cm m = Tr<S>::ld(u[(int64_t)k0 * pl + col]);
    Cm Q[D];
#pragma unroll
    for (int s = 0; s < D; ++s) Q[s] = Tr<S>::ld(u[(int64_t)min(k0 + 1 + s, nz + 1) * pl + col]);
    for (int kb = k0; kb < k1; kb += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) {
            const int k = kb + s;
            const int64_t p = (int64_t)min(k, nz) * pl + col;
            const Cm up = Q[s];
            const int64_t pw = (NEU && j == 1) ? p : p - 1, pe = (NEU && j == nx) ? p : p + 1;
            const int64_t ps = (NEU && i == 1) ? p : p - px, pn = (NEU && i == ny) ? p : p + px;
            const Cm dnv = (NEU && k == 1) ? m : dn, upv = (NEU && k >= nz) ? m : up;
            const Cm sm = ((Tr<S>::ld(u[pw]) + Tr<S>::ld(u[pe])) +
                           wy * (Tr<S>::ld(u[ps]) + Tr<S>::ld(u[pn]))) +
                          wz * (dnv + upv);
            const Cm t = (sm + Tr<S>::ld(b[p])) - dg * m;
            // planes k >= k1 land at or past the record count and are dropped
            tb_store(Tr<S>::st(m + c * t), rs, (int)(((int64_t)(k - k0) * pl + col) * (int64_t)sizeof(S)));
            dn = m;
            m = up;
            Q[s] = Tr<S>::ld(u[(int64_t)min(k + 1 + D, nz + 1) * pl + col]);
        }
    }
}

// One step of a variable-coefficient operator (Jacobi-scaled weights in g.w, Sec. 5.3's
// operators): s = (wW W + wE E) + (wS S + wN N) [+ (wD D + wU U)], t = (s + b) - u,
// u' = u + c t at every interior point whose mask is 0; masked points keep their value.
// One thread per interior point, binary64.
__global__ __launch_bounds__(256) void k_op_sweep(const double* __restrict__ u, double* __restrict__ o,
                                                  const double* __restrict__ b, Geo g, double c)
{
    const int j = blockIdx.x * 64 + threadIdx.x + 1;
    const int i = blockIdx.y * 4 + threadIdx.y + 1;
    const int k = g.ndim == 3 ? (int)blockIdx.z + 1 : 0;
    if (j > g.nx || i > g.ny) return;
    const int64_t pl = g.px * g.py;
    const int64_t p = (int64_t)k * pl + (int64_t)i * g.px + j;
    if (g.mask && g.mask[p]) {
        o[p] = u[p];
        return;
    }
    double s = (g.w[0][p] * u[p - 1] + g.w[1][p] * u[p + 1]) + (g.w[2][p] * u[p - g.px] + g.w[3][p] * u[p + g.px]);
    if (g.ndim == 3) s = s + (g.w[4][p] * u[p - pl] + g.w[5][p] * u[p + pl]);
    const double t = (s + b[p]) - u[p];
    o[p] = u[p] + c * t;
}

// ------------------------------------------------------------------ residuals

template <class S>
__device__ __forceinline__ double ldz(const S* u, int64_t p, bool zero)
{
    return zero ? 0.0 : (double)Tr<S>::ld(u[p]);
}

// r at interior point p (binary64).  With zero_int, interior values of u read as 0.
template <class S>
__device__ __forceinline__ double res_at(const S* u, const double* b64, int64_t p, int64_t px,
                                         int64_t pl, int ndim, int i, int j, int k, const Geo& g,
                                         bool zi)
{
    if (g.op) {
        // variable-coefficient operator: the Jacobi-scaled residual, 0 at masked points; with
        // zi the free interior points read as 0 (masked points and the ring keep their values)
        if (g.mask && g.mask[p]) return 0.0;
        auto rd = [&](int64_t q, bool interior) {
            const bool z = zi && interior && !(g.mask && g.mask[q]);
            return z ? 0.0 : (double)Tr<S>::ld(u[q]);
        };
        double s = (g.w[0][p] * rd(p - 1, j - 1 >= 1) + g.w[1][p] * rd(p + 1, j + 1 <= g.nx)) +
                   (g.w[2][p] * rd(p - px, i - 1 >= 1) + g.w[3][p] * rd(p + px, i + 1 <= g.ny));
        if (ndim == 3) s = s + (g.w[4][p] * rd(p - pl, k - 1 >= 1) + g.w[5][p] * rd(p + pl, k + 1 <= g.nz));
        return (s + b64[p]) - (zi ? 0.0 : (double)Tr<S>::ld(u[p]));
    }
    // Neumann: a neighbour across the boundary is the point itself (read as 0 with zi too)
    const bool neu = g.bc == 1;
    const bool inl = j - 1 >= 1, inr = j + 1 <= g.nx, ins = i - 1 >= 1, inn = i + 1 <= g.ny;
    const int64_t pw = (neu && !inl) ? p : p - 1, pe = (neu && !inr) ? p : p + 1;
    const int64_t ps = (neu && !ins) ? p : p - px, pn = (neu && !inn) ? p : p + px;
    const bool zl = zi && (inl || neu), zr = zi && (inr || neu);
    const bool zs = zi && (ins || neu), zn = zi && (inn || neu);
    double s = (ldz(u, pw, zl) + ldz(u, pe, zr)) + g.wy * (ldz(u, ps, zs) + ldz(u, pn, zn));
    if (ndim == 3) {
        const bool ind = k - 1 >= 1, inu = k + 1 <= g.nz;
        const int64_t pd = (neu && !ind) ? p : p - pl, pu = (neu && !inu) ? p : p + pl;
        const bool zd = zi && (ind || neu), zu = zi && (inu || neu);
        s = s + g.wz * (ldz(u, pd, zd) + ldz(u, pu, zu));
    }
    return (s + b64[p]) - g.dg * ldz(u, p, zi);
}

template <class S>
__global__ __launch_bounds__(256) void k_residual(const S* __restrict__ u, const double* __restrict__ b64,
                                                  Geo g, int zero_int, double* __restrict__ partials)
{
    const int64_t lines = g.ny * (g.ndim == 3 ? g.nz : 1);
    const int64_t pl = g.px * g.py;
    double s = 0.0, m = 0.0;
    const int rpb = res_rows(lines);
    const int64_t q0 = (int64_t)blockIdx.x * rpb;
    for (int64_t q = q0; q < min(q0 + rpb, lines); ++q) {
        const int i = (int)(q % g.ny) + 1;
        const int k = (g.ndim == 3) ? (int)(q / g.ny) + 1 : 0;
        const int64_t rowp = (int64_t)k * pl + (int64_t)i * g.px;
        for (int j = threadIdx.x + 1; j <= g.nx; j += 256) {
            double r = res_at(u, b64, rowp + j, g.px, pl, g.ndim, i, j, k, g, zero_int != 0);
            s = s + r * r;
            nanmax(m, fabs(r));
        }
    }
    block_reduce(s, m);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s;
        partials[2 * blockIdx.x + 1] = m;
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_residual_to_lo(const double* __restrict__ u,
                                                        const double* __restrict__ b64,
                                                        S* __restrict__ rlo, Geo g,
                                                        double* __restrict__ partials)
{
    const int64_t lines = g.ny * (g.ndim == 3 ? g.nz : 1);
    const int64_t pl = g.px * g.py;
    double s = 0.0, m = 0.0;
    const int rpb = res_rows(lines);
    const int64_t q0 = (int64_t)blockIdx.x * rpb;
    for (int64_t q = q0; q < min(q0 + rpb, lines); ++q) {
        const int i = (int)(q % g.ny) + 1;
        const int k = (g.ndim == 3) ? (int)(q / g.ny) + 1 : 0;
        const int64_t rowp = (int64_t)k * pl + (int64_t)i * g.px;
        for (int j = threadIdx.x + 1; j <= g.nx; j += 256) {
            double r = res_at(u, b64, rowp + j, g.px, pl, g.ndim, i, j, k, g, false);
            rlo[rowp + j] = Tr<S>::from64(r);
            s = s + r * r;
            nanmax(m, fabs(r));
        }
    }
    block_reduce(s, m);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s;
        partials[2 * blockIdx.x + 1] = m;
    }
}

// r = b64 - A u (binary64) written to a user array (dense layout, ring included) with 0 on
// the ring; one thread per user element.
__global__ __launch_bounds__(256) void k_residual_out(const double* __restrict__ u, const double* __restrict__ b64,
                                                      double* __restrict__ r, Geo g)
{
    const int64_t nxw = g.nx + 2, nyw = g.ny + 2, nzw = (g.ndim == 3 ? g.nz + 2 : 1);
    const int64_t n = nxw * nyw * nzw;
    const int64_t pl = g.px * g.py;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(idx % nxw);
        const int64_t t = idx / nxw;
        const int i = (int)(t % nyw);
        const int k = (g.ndim == 3) ? (int)(t / nyw) : 0;
        const bool inside = j >= 1 && j <= g.nx && i >= 1 && i <= g.ny && (g.ndim != 3 || (k >= 1 && k <= g.nz));
        r[idx] = inside ? res_at(u, b64, (int64_t)k * pl + (int64_t)i * g.px + j, g.px, pl, g.ndim, i, j, k, g, false)
                        : 0.0;
    }
}

// One binary64 sweep that also yields the residual of the state it starts from: at every
// interior point r = b - A u is formed as res_at forms it, which is the sweep's correction
// term t bit for bit (same association, and the fused x - 4m of the blocked kernels is exact),
// and the point is updated to u + c r (points under an operator's mask keep their value).  The
// blocks cover the lines of k_residual in its order and its block reduction, so the partial
// sums, and the norms k_reduce_final makes of them, equal those of a separate residual
// evaluation: a cycle's check comes out of the cycle's first sweep (Sec. 2's stopping rule).
__global__ __launch_bounds__(256) void k_sweep_residual(const double* __restrict__ u, double* __restrict__ o,
                                                        const double* __restrict__ b64, Geo g, double c,
                                                        double* __restrict__ partials)
{
    const int64_t lines = g.ny * (g.ndim == 3 ? g.nz : 1);
    const int64_t pl = g.px * g.py;
    double s = 0.0, m = 0.0;
    const int rpb = res_rows(lines);
    const int64_t q0 = (int64_t)blockIdx.x * rpb;
    for (int64_t q = q0; q < min(q0 + rpb, lines); ++q) {
        const int i = (int)(q % g.ny) + 1;
        const int k = (g.ndim == 3) ? (int)(q / g.ny) + 1 : 0;
        const int64_t rowp = (int64_t)k * pl + (int64_t)i * g.px;
        for (int j = threadIdx.x + 1; j <= g.nx; j += 256) {
            const int64_t p = rowp + j;
            const double r = res_at(u, b64, p, g.px, pl, g.ndim, i, j, k, g, false);
            const double up = u[p];
            o[p] = (g.op && g.mask && g.mask[p]) ? up : up + c * r;
            s = s + r * r;
            nanmax(m, fabs(r));
        }
    }
    block_reduce(s, m);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = s;
        partials[2 * blockIdx.x + 1] = m;
    }
}

// Deterministic final reduction: thread t folds partials t, t+256, ... in order.
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ partials, int n,
                                                      double* __restrict__ result)
{
    double s = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        s = s + partials[2 * i];
        nanmax(m, partials[2 * i + 1]);
    }
    block_reduce(s, m);
    if (threadIdx.x == 0) {
        result[0] = s;
        result[1] = m;
    }
}

template <class S>
__global__ __launch_bounds__(256) void k_update(double* __restrict__ u, const S* __restrict__ d, Geo g)
{
    const int64_t planes = (g.ndim == 3 ? g.nz : 1);
    const int64_t n = planes * g.ny * g.nx;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = idx % g.nx + 1;
        int64_t t = idx / g.nx;
        int64_t i = t % g.ny + 1;
        int64_t k = (g.ndim == 3) ? t / g.ny + 1 : 0;
        int64_t p = (k * g.py + i) * g.px + j;
        u[p] = u[p] + (double)Tr<S>::ld(d[p]);
    }
}

// Adjoint outputs, one thread per point of the user (dense, ring included) layout:
// df = hh * lam on the interior; dg = grad_u + (axis weight) * lam at the reading interior
// cell on the ring.
__global__ __launch_bounds__(256) void k_adjoint_out(const double* __restrict__ lam,
                                                     const double* __restrict__ gu, double hh,
                                                     double* __restrict__ df, double* __restrict__ dg,
                                                     Geo g)
{
    const int64_t nxw = g.nx + 2, nyw = g.ny + 2, nzw = (g.ndim == 3 ? g.nz + 2 : 1);
    const int64_t n = nxw * nyw * nzw;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx % nxw;
        const int64_t t = idx / nxw;
        const int64_t i = t % nyw;
        const int64_t k = (g.ndim == 3) ? t / nyw : 0;
        const bool ix = j >= 1 && j <= g.nx, iy = i >= 1 && i <= g.ny;
        const bool iz = (g.ndim == 3) ? (k >= 1 && k <= g.nz) : true;
        const int64_t p = (k * g.py + i) * g.px + j;
        if (df) df[idx] = (ix && iy && iz) ? hh * lam[p] : 0.0;
        if (dg) {
            double v = 0.0;
            // a ring cell is read by exactly one stencil when it lies outside the box along
            // exactly one axis; its reader is the adjacent interior cell along that axis,
            // which weighs it with that axis's weight
            const int outs = (!ix) + (!iy) + ((g.ndim == 3) && !iz);
            if (outs == 1) {
                int64_t jj = j, ii = i, kk = k;
                double wa = 1.0;
                if (!ix) jj = (j == 0) ? 1 : g.nx;
                if (!iy) {
                    ii = (i == 0) ? 1 : g.ny;
                    wa = g.wy;
                }
                if (g.ndim == 3 && !iz) {
                    kk = (k == 0) ? 1 : g.nz;
                    wa = g.wz;
                }
                v = wa * lam[(kk * g.py + ii) * g.px + jj];
            }
            // the ring of u is g itself: its own gradient passes straight through
            dg[idx] = (ix && iy && iz) ? 0.0 : v + gu[idx];
        }
    }
}

// ------------------------------------------------------------------ launchers

static dim3 grid1d(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

static int64_t field_rows(const Geo& g) { return (g.ndim == 3 ? g.nz + 2 : 1) * g.py; }


hipError_t launch_copy_in(Fmt f, const double* user, void* field, const Geo& g, hipStream_t s)
{
    int64_t n = field_rows(g) * (g.nx + 2);
    SRJ_DISPATCH(f, hipLaunchKernelGGL(k_copy_in<S>, grid1d(n), dim3(256), 0, s, user, (S*)field, g));
    return hipGetLastError();
}

hipError_t launch_copy_out(Fmt f, const void* field, double* user, const Geo& g, hipStream_t s)
{
    int64_t n = (g.ndim == 3 ? g.nz : 1) * g.ny * g.nx;
    SRJ_DISPATCH(f, hipLaunchKernelGGL(k_copy_out<S>, grid1d(n), dim3(256), 0, s, (const S*)field, user, g));
    return hipGetLastError();
}

hipError_t launch_rhs(Fmt f, const double* uf, double hh, void* blo, double* b64, const Geo& g,
                      hipStream_t s)
{
    int64_t n = (g.ndim == 3 ? g.nz : 1) * g.ny * g.nx;
    SRJ_DISPATCH(f, hipLaunchKernelGGL(k_rhs<S>, grid1d(n), dim3(256), 0, s, uf, hh, (S*)blo, b64, g));
    return hipGetLastError();
}

hipError_t launch_zero(Fmt f, void* field, const Geo& g, hipStream_t s)
{
    int64_t n = field_rows(g) * g.px;
    SRJ_DISPATCH(f, hipLaunchKernelGGL(k_zero<S>, grid1d(n), dim3(256), 0, s, (S*)field, n));
    return hipGetLastError();
}

hipError_t launch_sweep_unfused(Fmt f, const void* in, void* out, const void* b, const Geo& g,
                                double c, hipStream_t s)
{
    if (g.op) {
        if (f != FMT_F64) return hipErrorInvalidValue;
        dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4), (unsigned)(g.ndim == 3 ? g.nz : 1));
        hipLaunchKernelGGL(k_op_sweep, grid, dim3(64, 4), 0, s, (const double*)in, (double*)out, (const double*)b, g,
                           c);
        return hipGetLastError();
    }
    if (g.ndim == 2) {
        dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + 3) / 4));
        if (g.bc == 1)
            SRJ_DISPATCH(f, hipLaunchKernelGGL((k_sweep2d<S, true>), grid, dim3(64, 4), 0, s, (const S*)in, (S*)out,
                                               (const S*)b, g.px, (int)g.nx, (int)g.ny, g.wy, g.dg, c))
        else
            SRJ_DISPATCH(f, hipLaunchKernelGGL((k_sweep2d<S, false>), grid, dim3(64, 4), 0, s, (const S*)in,
                                               (S*)out, (const S*)b, g.px, (int)g.nx, (int)g.ny, g.wy, g.dg, c))
    } else {
        // 64 x 4 threads per block, runs of 32 z planes, 2 planes loaded ahead
        constexpr int kZrun = 32, kBy = 4;
        // the run's byte offsets (plus the planes loaded ahead) stay below 2^31
        const int64_t zmax = ((int64_t)1 << 31) / ((int64_t)fmt_size(f) * g.px * g.py) - 6;
        const int zrun = (int)std::max<int64_t>(1, std::min<int64_t>(kZrun, zmax));
        dim3 grid((unsigned)((g.nx + 63) / 64), (unsigned)((g.ny + kBy - 1) / kBy), (unsigned)((g.nz + zrun - 1) / zrun));
        dim3 blk(64, kBy);
        if (g.bc == 1)
            SRJ_DISPATCH(f, hipLaunchKernelGGL((k_sweep3d<S, 2, true>), grid, blk, 0, s, (const S*)in, (S*)out,
                                               (const S*)b, g.px, g.py, (int)g.nx, (int)g.ny, (int)g.nz, zrun, g.wy,
                                               g.wz, g.dg, c))
        else
            SRJ_DISPATCH(f, hipLaunchKernelGGL((k_sweep3d<S, 2, false>), grid, blk, 0, s, (const S*)in, (S*)out,
                                               (const S*)b, g.px, g.py, (int)g.nx, (int)g.ny, (int)g.nz, zrun, g.wy,
                                               g.wz, g.dg, c))
    }
    return hipGetLastError();
}

int residual_blocks(const Geo& g)
{
    int64_t lines = g.ny * (g.ndim == 3 ? g.nz : 1);
    const int rpb = res_rows(lines);
    return (int)((lines + rpb - 1) / rpb);
}

hipError_t launch_residual(Fmt f, const void* u, const double* b64, const Geo& g, int zero_interior,
                           double* partials, double* result, hipStream_t s)
{
    int nb = residual_blocks(g);
    SRJ_DISPATCH(f, hipLaunchKernelGGL(k_residual<S>, dim3(nb), dim3(256), 0, s, (const S*)u, b64, g,
                                       zero_interior, partials));
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, partials, nb, result);
    return hipGetLastError();
}

hipError_t launch_sweep_residual(const double* u, double* out, const double* b64, const Geo& g, double c,
                                 double* partials, double* result, hipStream_t s)
{
    const int nb = residual_blocks(g);
    hipLaunchKernelGGL(k_sweep_residual, dim3(nb), dim3(256), 0, s, u, out, b64, g, c, partials);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, partials, nb, result);
    return hipGetLastError();
}

hipError_t launch_residual_to_lo(Fmt f, const double* u64, const double* b64, void* rlo, const Geo& g,
                                 double* partials, double* result, hipStream_t s)
{
    int nb = residual_blocks(g);
    SRJ_DISPATCH(f, hipLaunchKernelGGL(k_residual_to_lo<S>, dim3(nb), dim3(256), 0, s, u64, b64, (S*)rlo, g,
                                       partials));
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(256), 0, s, partials, nb, result);
    return hipGetLastError();
}

hipError_t launch_residual_out(const double* u64, const double* b64, double* r_user, const Geo& g, hipStream_t s)
{
    int64_t n = (g.ndim == 3 ? g.nz + 2 : 1) * (g.ny + 2) * (g.nx + 2);
    hipLaunchKernelGGL(k_residual_out, grid1d(n), dim3(256), 0, s, u64, b64, r_user, g);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_op_setup(const double* __restrict__ coef, const uint8_t* __restrict__ mu,
                                                  Geo g, double* w0, double* w1, double* w2, double* w3, double* w4,
                                                  double* w5, double* __restrict__ ap, uint8_t* __restrict__ mask)
{
    const int64_t nxw = g.nx + 2, nyw = g.ny + 2, nzw = (g.ndim == 3 ? g.nz + 2 : 1);
    const int64_t n = nxw * nyw * nzw;
    double* w[6] = {w0, w1, w2, w3, w4, w5};
    const int nnb = 2 * g.ndim;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx % nxw, t = idx / nxw, i = t % nyw, k = t / nyw;
        const int64_t p = (k * g.py + i) * g.px + j;
        const bool inside = j >= 1 && j <= g.nx && i >= 1 && i <= g.ny && (g.ndim != 3 || (k >= 1 && k <= g.nz));
        const double a = coef[idx];
        for (int m = 0; m < nnb; ++m) w[m][p] = inside ? coef[(int64_t)(m + 1) * n + idx] / a : 0.0;
        ap[p] = inside ? a : 0.0;
        if (mask) mask[p] = mu ? mu[idx] : 0;
    }
}

__global__ __launch_bounds__(256) void k_op_rhs(const double* __restrict__ uf, const double* __restrict__ ap,
                                                double* __restrict__ b, Geo g)
{
    const int64_t planes = (g.ndim == 3 ? g.nz : 1);
    const int64_t n = planes * g.ny * g.nx;
    const int64_t w = g.nx + 2;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = idx % g.nx + 1, t = idx / g.nx, i = t % g.ny + 1;
        const int64_t k = (g.ndim == 3) ? t / g.ny + 1 : 0;
        const int64_t row = k * g.py + i, p = row * g.px + j;
        const bool fixed = g.mask && g.mask[p];
        b[p] = fixed ? 0.0 : uf[row * w + j] / ap[p];
    }
}

hipError_t launch_op_setup(const double* coef, const uint8_t* mask_user, double* const* w, double* ap,
                           uint8_t* mask, const Geo& g, hipStream_t s)
{
    int64_t n = (g.ndim == 3 ? g.nz + 2 : 1) * (g.ny + 2) * (g.nx + 2);
    double* ww[6] = {w[0], w[1], w[2], w[3], g.ndim == 3 ? w[4] : w[0], g.ndim == 3 ? w[5] : w[0]};
    hipLaunchKernelGGL(k_op_setup, grid1d(n), dim3(256), 0, s, coef, mask_user, g, ww[0], ww[1], ww[2], ww[3], ww[4],
                       ww[5], ap, mask);
    return hipGetLastError();
}

hipError_t launch_op_rhs(const double* user_f, const double* ap, double* b64, const Geo& g, hipStream_t s)
{
    int64_t n = (g.ndim == 3 ? g.nz : 1) * g.ny * g.nx;
    hipLaunchKernelGGL(k_op_rhs, grid1d(n), dim3(256), 0, s, user_f, ap, b64, g);
    return hipGetLastError();
}

hipError_t launch_adjoint_out(const double* lam, const double* grad_u, double hh, double* df, double* dg,
                              const Geo& g, hipStream_t s)
{
    int64_t n = (g.ndim == 3 ? g.nz + 2 : 1) * (g.ny + 2) * (g.nx + 2);
    hipLaunchKernelGGL(k_adjoint_out, grid1d(n), dim3(256), 0, s, lam, grad_u, hh, df, dg, g);
    return hipGetLastError();
}

hipError_t launch_update(Fmt f, double* u64, const void* d, const Geo& g, hipStream_t s)
{
    int64_t n = (g.ndim == 3 ? g.nz : 1) * g.ny * g.nx;
    SRJ_DISPATCH(f, hipLaunchKernelGGL(k_update<S>, grid1d(n), dim3(256), 0, s, u64, (const S*)d, g));
    return hipGetLastError();
}

}  // namespace srj
