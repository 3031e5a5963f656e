// Register-pipelined 2D tile of the temporally blocked SRJ sweep (shared by the single-grid
// and the batched kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "formats.h"

namespace srj {

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

// Copy of a (uniform) integer into a vector register.  The row-validity test below is then
// evaluated per lane and becomes a select; evaluated on a scalar it is compiled into jumps
// around the arithmetic of every level.  Register move only, no memory access.
__device__ __forceinline__ int vcopy(int x)
{
    int y;
    asm("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
    return y;
}

// One wave computes Tact <= T consecutive sweeps (coefficients cf[0..Tact)) of the tile
// (strip st, segment sg) of an nx x ny grid: strip st covers columns x0 .. x0 + 64C - 1 with
// x0 = 1 + st*SW - T (SW = 64C - 2T output columns per strip); segment sg outputs rows
// y0 .. y1-1.  At step r the wave takes row r (level 0) and computes level l for row r - l,
// l = 1..T, from level l-1 rows r-l-1, r-l, r-l+1; the value of level T for row r - T is
// stored if that row belongs to the segment.  Levels above Tact pass values through
// unchanged.  Ring rows/columns never change; lanes or rows outside the grid read clamped
// (in-bounds) addresses and are never updated or stored, and only points whose dependence
// cone lies inside the loaded window are stored.  The step loop is free of branches so
// that the D row loads in flight (register slots named statically by unrolling the loop D
// times) overlap D steps of arithmetic.
template <class S, int T, int C, int D>
__device__ __forceinline__ void tb_tile(const S* __restrict__ uin, S* __restrict__ uout,
                                        const S* __restrict__ bb, int64_t px, int nx, int ny,
                                        const typename Tr<S>::C (&cf)[T], int Tact, int st, int sg,
                                        int H)
{
    using Cm = typename Tr<S>::C;
    constexpr int SW = 64 * C - 2 * T;
    const int lane = threadIdx.x & 63;
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
            const int rv = vcopy(r);
            Cm in[C];
#pragma unroll
            for (int c = 0; c < C; ++c) in[c] = U[s][c];
#pragma unroll
            for (int l = 1; l <= T; ++l) {
                const int jv = rv - l;
                const bool rowok = (jv >= 1) & (jv <= ny) & (l <= Tact);
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
                    Cm v = Tr<S>::ld(Tr<S>::st(m + cf[l - 1] * t));
                    // v is always computed: an empty register constraint keeps the compiler
                    // from sinking its arithmetic under a branch
                    asm("" : "+v"(v));
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

}  // namespace srj
