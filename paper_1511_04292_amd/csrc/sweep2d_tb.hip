// Temporally blocked 2D SRJ sweep for gfx950 (CDNA4, wave64).
//
// T consecutive scheduled sweeps (Sec. 2; each step as in Sec. 3.1, Eq. 2nd-order_CD,
// evaluated with the association and rounding of the unfused kernel, so the result is
// bit-identical to T unfused sweeps) are applied in one launch.  Each wavefront owns a
// strip of 64*C columns (C per lane) and a segment of rows, streams the rows from top to
// bottom and keeps T time levels of a 3-row window in registers: one HBM read of u and b
// and one write of u serve T sweeps.  Horizontal neighbours cross lanes by DPP lane
// shifts; no LDS and no barriers are needed because every wave is independent (strips
// overlap by T columns on each side, segments by T rows, the overlap being recomputed).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>

#include "formats.h"
#include "kernels.h"

namespace srj {

// --------------------------------------------------- temporally blocked 2D sweeps

template <int T> struct CoefsT {
    double c[T];
};

// Lane shifts through DPP (wave_shr:1 / wave_shl:1): lane i receives lane i-1 (resp. i+1).
// The wave's edge lanes receive 0; their results are never stored.
__device__ __forceinline__ float dpp_from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double dpp_from_left(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double dpp_from_right(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Wave layout: strip `st` covers columns x0 .. x0 + 64C - 1 with x0 = 1 + st*SW - T
// (SW = 64C - 2T output columns per strip); segment `sg` outputs rows y0 .. y1-1.
// At step r the wave takes row r (level 0) and computes level l for row r - l,
// l = 1..T, from level l-1 rows r-l-1, r-l, r-l+1; the value of level T for row r - T
// is stored if that row belongs to the segment.  Ring rows/columns never change; lanes
// or rows outside the grid read clamped (in-bounds) addresses and are never updated or
// stored, and only points whose dependence cone lies inside the loaded window are
// stored.  The step loop is free of branches so that the D row loads in flight (register
// slots named statically by unrolling the loop D times) overlap D steps of arithmetic.
// Optionally blocks are remapped so that each of the 8 XCDs works on a contiguous band
// of tiles, keeping the overlapping halo reads of neighbouring waves in one L2.
template <class S, int T, int C, int D>
__global__ __launch_bounds__(256) void k_sweep2d_tb(const S* __restrict__ uin, S* __restrict__ uout,
                                                    const S* __restrict__ bb, int64_t px, int nx,
                                                    int ny, CoefsT<T> co, int nstrip, int nwaves,
                                                    int H, int remap)
{
    using Cm = typename Tr<S>::C;
    constexpr int SW = 64 * C - 2 * T;
    const int lane = threadIdx.x & 63;
    const int nblk = (int)gridDim.x;  // a multiple of 8 (padded by the launcher)
    const int blk = remap ? (int)(blockIdx.x & 7) * (nblk >> 3) + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
    const int wid = blk * 4 + (threadIdx.x >> 6);
    if (wid >= nwaves) return;
    const int st = wid % nstrip;
    const int sg = wid / nstrip;
    const int64_t x0 = 1 + (int64_t)st * SW - T + (int64_t)lane * C;
    const int y0 = 1 + sg * H;
    const int y1 = min(y0 + H, ny + 1);
    const int rb = max(0, y0 - T);
    const int rl = y1 - 1 + T;

    bool upd[C], outc[C];
    int64_t xc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t x = x0 + c;
        const int off = lane * C + c;
        upd[c] = (x >= 1 && x <= (int64_t)nx);
        outc[c] = upd[c] && off >= T && off < 64 * C - T;
        xc[c] = x < 0 ? 0 : (x > (int64_t)nx + 1 ? (int64_t)nx + 1 : x);
    }
    Cm cf[T];
#pragma unroll
    for (int l = 0; l < T; ++l) cf[l] = (Cm)co.c[l];

    Cm p1[T][C], p2[T][C], bq[T][C];
#pragma unroll
    for (int l = 0; l < T; ++l)
#pragma unroll
        for (int c = 0; c < C; ++c) p1[l][c] = p2[l][c] = bq[l][c] = (Cm)0;

    // in-bounds loads of row r (clamped to the last ring row)
    auto load_row = [&](int r, Cm* vu, Cm* vb) {
        const int64_t rowp = (int64_t)min(r, ny + 1) * px;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            vu[c] = Tr<S>::ld(uin[rowp + xc[c]]);
            vb[c] = Tr<S>::ld(bb[rowp + xc[c]]);
        }
    };

    Cm U[D][C], B[D][C];
#pragma unroll
    for (int s = 0; s < D; ++s) load_row(rb + s, U[s], B[s]);

    const int nsteps = rl - rb + 1;
    for (int r0 = rb; r0 < rb + nsteps; r0 += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) {
            const int r = r0 + s;
            Cm in[C];
#pragma unroll
            for (int c = 0; c < C; ++c) in[c] = U[s][c];
#pragma unroll
            for (int l = 1; l <= T; ++l) {
                const int j = r - l;
                const bool rowok = (j >= 1) & (j <= ny);
                const Cm wn = dpp_from_left(p1[l - 1][C - 1]);
                const Cm en = dpp_from_right(p1[l - 1][0]);
                Cm out[C];
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const Cm W = (c == 0) ? wn : p1[l - 1][c - 1];
                    const Cm E = (c == C - 1) ? en : p1[l - 1][c + 1];
                    const Cm m = p1[l - 1][c];
                    const Cm sm = (W + E) + (p2[l - 1][c] + in[c]);
                    const Cm t = (sm + bq[l - 1][c]) - (Cm)4 * m;
                    const Cm v = Tr<S>::ld(Tr<S>::st(m + cf[l - 1] * t));
                    out[c] = (rowok && upd[c]) ? v : m;
                }
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    p2[l - 1][c] = p1[l - 1][c];
                    p1[l - 1][c] = in[c];
                    in[c] = out[c];
                }
            }
            const int j = r - T;
            const bool rowout = (j >= y0) & (j < y1);
            S* po = uout + (int64_t)j * px + x0;
#pragma unroll
            for (int c = 0; c < C; ++c)
                if (rowout && outc[c]) po[c] = Tr<S>::st(in[c]);
#pragma unroll
            for (int l = T - 1; l > 0; --l)
#pragma unroll
                for (int c = 0; c < C; ++c) bq[l][c] = bq[l - 1][c];
#pragma unroll
            for (int c = 0; c < C; ++c) bq[0][c] = B[s][c];
            load_row(r + D, U[s], B[s]);
        }
    }
}

static int env_int(const char* name, int dflt)
{
    const char* v = getenv(name);
    return v ? atoi(v) : dflt;
}

template <class S, int T, int C, int D>
static void tb2d(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int H, hipStream_t s)
{
    constexpr int SW = 64 * C - 2 * T;
    static const int remap = env_int("SRJ_TB_XCD_REMAP", 1);  // tuning knob, default on
    CoefsT<T> ct;
    for (int l = 0; l < T; ++l) ct.c[l] = co.c[l];
    const int nstrip = (int)((g.nx + SW - 1) / SW);
    const int nseg = (int)((g.ny + H - 1) / H);
    const int nwaves = nstrip * nseg;
    const int nblk = ((nwaves + 3) / 4 + 7) / 8 * 8;
    hipLaunchKernelGGL((k_sweep2d_tb<S, T, C, D>), dim3(nblk), dim3(256), 0, s, in, out, b, g.px,
                       (int)g.nx, (int)g.ny, ct, nstrip, nwaves, H, remap);
}

template <class S, int C, int D>
static void tb2d_T(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int T, int H, hipStream_t s)
{
    switch (T) {
    case 1: tb2d<S, 1, C, D>(in, out, b, g, co, H, s); break;
    case 2: tb2d<S, 2, C, D>(in, out, b, g, co, H, s); break;
    case 3: tb2d<S, 3, C, D>(in, out, b, g, co, H, s); break;
    case 4: tb2d<S, 4, C, D>(in, out, b, g, co, H, s); break;
    case 5: tb2d<S, 5, C, D>(in, out, b, g, co, H, s); break;
    case 6: tb2d<S, 6, C, D>(in, out, b, g, co, H, s); break;
    case 7: tb2d<S, 7, C, D>(in, out, b, g, co, H, s); break;
    default: tb2d<S, 8, C, D>(in, out, b, g, co, H, s); break;
    }
}

template <class S>
static void tb2d_dispatch(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int T,
                          int H, hipStream_t s)
{
    constexpr int C = 2;
    static const int pf = env_int("SRJ_TB_PREFETCH", 4);
    if (pf == 1) {
        tb2d_T<S, C, 1>(in, out, b, g, co, T, H, s);
    } else if (pf == 2) {
        tb2d_T<S, C, 2>(in, out, b, g, co, T, H, s);
    } else {
        tb2d_T<S, C, 4>(in, out, b, g, co, T, H, s);
    }
}

hipError_t launch_sweep_fused(Fmt f, const void* in, void* out, const void* b, const Geo& g,
                              const Coefs& co, int T, int H, hipStream_t s)
{
    if (g.ndim != 2 || T < 1 || T > kMaxFuse || H < 1) return hipErrorInvalidValue;
    SRJ_DISPATCH(f, tb2d_dispatch<S>((const S*)in, (S*)out, (const S*)b, g, co, T, H, s));
    return hipGetLastError();
}


}  // namespace srj
