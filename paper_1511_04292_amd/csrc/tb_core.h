// Register-pipelined 2D tile of the temporally blocked SRJ sweep (shared by the single-grid
// and the batched kernels).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "formats.h"

namespace srj {

// Lane shifts through DPP (wave_shr:1 / wave_shl:1): lane i receives lane i-1 (resp. i+1).
// The wave's edge lanes have no source and receive 0 (bound_ctrl); their results are never
// stored.
__device__ __forceinline__ int dpp_shr1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int dpp_shl1(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ float dpp_from_left(float v) { return __int_as_float(dpp_shr1(__float_as_int(v))); }
__device__ __forceinline__ float dpp_from_right(float v) { return __int_as_float(dpp_shl1(__float_as_int(v))); }
__device__ __forceinline__ double dpp_from_left(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_shr1((int)(b & 0xffffffffll));
    const int hi = dpp_shr1((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double dpp_from_right(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_shl1((int)(b & 0xffffffffll));
    const int hi = dpp_shl1((int)(b >> 32));
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

// Stores of the tile go through a raw buffer resource whose range check drops the stores of
// masked lanes and rows (their byte offset is pushed past the record count), so the step
// loop stores without branches and the compiler can keep the row loads of later steps in
// flight across it.
typedef unsigned int tb_u32x2 __attribute__((ext_vector_type(2)));
constexpr int kTbMasked = 0x40000000;  // offset added for a masked row; the record count stays below it

// HINT is the stores' cache-policy operand: 0 (plain) or kTbStoreNt (the non-temporal bit).
// Which launches take the hint was measured, alternating builds on one machine: the fused
// binary64 3D sweep always (512^3 at 4 sweeps: 921 against 944 us), the fused binary64 2D
// sweep when its three fields exceed the memory-side cache but fit in twice it (4096^2 at 10
// sweeps: 87.3 against 89.2 us; 2048^2, inside the cache, was 37% slower at one sweep per
// launch, 8192^2 to 32768^2 2-3% slower at ten); the 4- and 2-byte formats never (3-6% slower).
constexpr int kTbStoreNt = 2;

template <int HINT = 0>
__device__ __forceinline__ void tb_store(double v, __amdgpu_buffer_rsrc_t r, int off)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(tb_u32x2, v), r, off, 0, HINT);
}
template <int HINT = 0>
__device__ __forceinline__ void tb_store(float v, __amdgpu_buffer_rsrc_t r, int off)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, HINT);
}
template <int HINT = 0>
__device__ __forceinline__ void tb_store(bf16_t v, __amdgpu_buffer_rsrc_t r, int off)
{
    __builtin_amdgcn_raw_buffer_store_b16(v.v, r, off, 0, HINT);
}

// Two neighbouring elements x, x+1 of a row in one load (x odd: the pair is aligned to its
// size, since interior column 1 of every row is).
typedef double tb_d2 __attribute__((ext_vector_type(2)));
typedef float tb_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void tb_ld_pair(const double* p, double& a, double& b)
{
    const tb_d2 v = *reinterpret_cast<const tb_d2*>(p);
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void tb_ld_pair(const float* p, float& a, float& b)
{
    const tb_f2 v = *reinterpret_cast<const tb_f2*>(p);
    a = v.x;
    b = v.y;
}
__device__ __forceinline__ void tb_ld_pair(const bf16_t* p, float& a, float& b)
{
    const uint32_t w = *reinterpret_cast<const uint32_t*>(p);
    a = __uint_as_float(w << 16);
    b = __uint_as_float(w & 0xffff0000u);
}

// x - 4m with one rounding.  4m is exact in binary floating point (a power-of-two scale; the
// field's magnitudes are far from overflow), so the fused multiply-add returns the same value
// as the product followed by the subtraction, in one instruction instead of two.
__device__ __forceinline__ double tb_sub4(double x, double m) { return __builtin_fma(-4.0, m, x); }
__device__ __forceinline__ float tb_sub4(float x, float m) { return __builtin_fmaf(-4.0f, m, x); }

// Each value rounded to the storage format and back (the level's result as a sweep stores
// it).  BF16 rounds two values with one conversion instruction; the others are exact.
typedef __bf16 tb_bf2 __attribute__((ext_vector_type(2)));
template <class S, int N>
__device__ __forceinline__ void tb_round(typename Tr<S>::C (&v)[N])
{
    if constexpr (std::is_same<S, bf16_t>::value && N % 2 == 0) {
#pragma unroll
        for (int i = 0; i < N; i += 2) {
            const tb_f2 x = {v[i], v[i + 1]};
            const uint32_t w = __builtin_bit_cast(uint32_t, __builtin_convertvector(x, tb_bf2));
            v[i] = __uint_as_float(w << 16);
            v[i + 1] = __uint_as_float(w & 0xffff0000u);
        }
    } else {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] = Tr<S>::ld(Tr<S>::st(v[i]));
    }
}

constexpr int tb_lcm(int a, int b)
{
    int x = a, y = b;
    while (y) {
        const int t = x % y;
        x = y;
        y = t;
    }
    return a / x * b;
}

// Largest segment height whose store window (H rows of pitch px plus one strip) keeps the
// buffer record count below kTbMasked.
inline int tb_max_rows(int64_t px, int esize)
{
    const int64_t lim = ((int64_t)kTbMasked / esize - 256) / px;
    return (int)(lim < 1 ? 1 : (lim > (1 << 20) ? (1 << 20) : lim));
}

// Pipeline state of one wave: T time levels of a 3-row window (rows r-l-1 .. r-l+1 of level
// l-1 held as p2, p1 and the incoming value), the scaled source of the row each level works
// on (bq[l-1] = b of row r-l), and D rows of u and b in flight.
template <class Cm, int T, int C, int D>
struct TbRegs {
    Cm p1[T][C], p2[T][C], bq[T][C];
    Cm U[D][C], B[D][C];
};

// One step of the pipeline: level-0 row r arrives from slot s; levels 1..lmax are computed
// (lmax < T only while the pipeline fills: level l is first needed at step 2l of the tile);
// the value of level T for row r - dir*T is stored if that row is an output row of the tile.
// dir = +1 streams rows downwards (level l works on row r - l), -1 upwards (row r + l); the
// window then holds the rows in the other order and (S + N) is formed as (N + S), which is
// the same IEEE sum.
// MODE says what the step must check:
//   TB_CLEAN: every computed point is an interior point of the grid and all T levels apply,
//             so no selects;
//   TB_COLS:  every computed row is an interior row and all T levels apply; columns outside
//             the grid (the ring and beyond, fixed per lane) keep their values;
//   TB_FULL:  rows, columns and levels above Tact are all checked.
enum { TB_CLEAN = 0, TB_COLS = 1, TB_FULL = 2 };
template <class S, int T, int C, int D, int MODE, int HINT>
__device__ __forceinline__ void tb_step(TbRegs<typename Tr<S>::C, T, C, D>& R, int s, int lmax, int r,
                                        const typename Tr<S>::C (&cf)[T], const bool (&upd)[C], int ny,
                                        int Tact, int y0, int y1, int rowbytes, const int (&lanebase)[C],
                                        __amdgpu_buffer_rsrc_t rs, int dir)
{
    using Cm = typename Tr<S>::C;
    Cm in[C];
#pragma unroll
    for (int c = 0; c < C; ++c) in[c] = R.U[s][c];
    const int rv = MODE == TB_FULL ? vcopy(r) : 0;
    const int dv = MODE == TB_FULL ? vcopy(dir) : 0;
#pragma unroll
    for (int l = 1; l <= T; ++l) {
        if (l > lmax + 1) break;
        Cm out[C];
        if (l <= lmax) {
            const Cm wn = dpp_from_left(R.p1[l - 1][C - 1]);
            const Cm en = dpp_from_right(R.p1[l - 1][0]);
            bool rowok = true;
            if (MODE == TB_FULL) {
                const int jv = rv - dv * l;
                rowok = (jv >= 1) & (jv <= ny) & (l <= Tact);
            }
            Cm vs[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const Cm W = (c == 0) ? wn : R.p1[l - 1][c - 1];
                const Cm E = (c == C - 1) ? en : R.p1[l - 1][c + 1];
                const Cm m = R.p1[l - 1][c];
                const Cm sm = (W + E) + (R.p2[l - 1][c] + in[c]);
                const Cm t = tb_sub4(sm + R.bq[l - 1][c], m);
                vs[c] = m + cf[l - 1] * t;
            }
            tb_round<S>(vs);
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const Cm m = R.p1[l - 1][c];
                Cm v = vs[c];
                if (MODE == TB_CLEAN) {
                    out[c] = v;
                } else {
                    // v is always computed: an empty register constraint keeps the compiler
                    // from sinking its arithmetic under a branch
                    asm("" : "+v"(v));
                    out[c] = (rowok && upd[c]) ? v : m;
                }
            }
        }
#pragma unroll
        for (int c = 0; c < C; ++c) {
            R.p2[l - 1][c] = R.p1[l - 1][c];
            R.p1[l - 1][c] = in[c];
            if (l <= lmax) in[c] = out[c];
        }
    }
    if (lmax == T) {
        const int j = r - dir * T;
        const int rowpart = (j >= y0 && j < y1) ? (j - y0) * rowbytes : kTbMasked;
#pragma unroll
        for (int c = 0; c < C; ++c) tb_store<HINT>(Tr<S>::st(in[c]), rs, rowpart + lanebase[c]);
    }
#pragma unroll
    for (int l = T - 1; l > 0; --l)
#pragma unroll
        for (int c = 0; c < C; ++c) R.bq[l][c] = R.bq[l - 1][c];
#pragma unroll
    for (int c = 0; c < C; ++c) R.bq[0][c] = R.B[s][c];
}

// One wave computes Tact <= T consecutive sweeps (coefficients cf[0..Tact)) of the tile
// (strip st, segment sg) of an nx x ny grid: strip st covers columns x0 .. x0 + 64C - 1 with
// x0 = 1 + st*SW - T (SW = 64C - 2T output columns per strip); segment sg outputs rows
// y0 .. y1-1 (H rows, fewer in the last segment).  The wave streams rows y0-T .. y1-1+T:
// at step r it takes row r (level 0) and computes level l for row r - l, l = 1..T, from
// level l-1 rows r-l-1, r-l, r-l+1; the value of level T for row r - T is stored if that row
// belongs to the segment.  Levels above Tact pass values through unchanged.  Ring rows and
// columns never change; rows outside the grid read clamped (in-bounds) addresses and are
// never updated or stored, and only points whose dependence cone lies inside the loaded
// window are stored.  The first steps (pipeline fill) compute only the levels whose rows
// are needed; the rest of the step loop is free of branches so that the D row loads in
// flight (register slots named statically by unrolling the loop D times) overlap D steps
// of arithmetic.  H * px * sizeof(S) must not exceed what tb_max_rows allows.
template <class S, int T, int C, int D, int FILL, int STEADY, bool WIDE, int HINT>
__device__ __forceinline__ void tb_tile_body(const S* __restrict__ uin, S* __restrict__ uout,
                                             const S* __restrict__ bb, int64_t px, int nx, int ny,
                                             const typename Tr<S>::C (&cf)[T], int Tact, int st, int sg, int H,
                                             int dir)
{
    using Cm = typename Tr<S>::C;
    constexpr int SW = 64 * C - 2 * T;
    constexpr int F = (2 * T + D - 1) / D * D;  // fill steps, a whole number of slot rounds
    const int lane = threadIdx.x & 63;
    const int64_t xs = 1 + (int64_t)st * SW - T;  // first column of the strip
    const int64_t x0 = xs + (int64_t)lane * C;
    const int y0 = 1 + sg * H;
    const int y1 = min(y0 + H, ny + 1);
    const int rb = y0 - T;
    const int rl = y1 - 1 + T;
    const int r_first = dir > 0 ? rb : rl;
    const int nsteps = rl - rb + 1;

    bool upd[C];
    int64_t xc[C];
    int lanebase[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t x = x0 + c;
        const int off = lane * C + c;
        upd[c] = (x >= 1 && x <= (int64_t)nx);
        const bool outc = upd[c] && off >= T && off < 64 * C - T;
        lanebase[c] = off * (int)sizeof(S) + (outc ? 0 : (int)0x80000000);
        xc[c] = x < 0 ? 0 : (x > (int64_t)nx + 1 ? (int64_t)nx + 1 : x);
    }
    const int rowbytes = (int)(px * (int64_t)sizeof(S));
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void*)(uout + (int64_t)y0 * px + xs), (short)0, (int)((int64_t)H * rowbytes + 128 * (int)sizeof(S)),
        0x00020000);

    TbRegs<Cm, T, C, D> R;
#pragma unroll
    for (int l = 0; l < T; ++l)
#pragma unroll
        for (int c = 0; c < C; ++c) R.p1[l][c] = R.p2[l][c] = R.bq[l][c] = (Cm)0;

    // With two columns per lane and T even, a lane's columns x0, x0+1 start at an odd x and
    // are loaded as one pair.  Pairs left of the ring start at -1 and pairs right of it at
    // the last odd x <= nx+1: one element beyond the ring column on either side, inside the
    // field's allocation.  Such lanes then hold values that are not the ring's, but they are
    // never updated or stored, and the ring lanes they feed keep their values.
    constexpr bool kPairs = (C == 2) && (T % 2 == 0);
    int64_t xpair = x0;
    if (kPairs) {
        const int64_t xlast = ((nx + 1) & 1) ? (int64_t)nx + 1 : (int64_t)nx;
        xpair = x0 < -1 ? -1 : (x0 > xlast ? xlast : x0);
    }

    // in-bounds loads of row r (clamped to the ring rows)
    auto load_row = [&](int r, Cm* vu, Cm* vb) {
        const int64_t rowp = (int64_t)max(0, min(r, ny + 1)) * px;
        if constexpr (kPairs) {
            tb_ld_pair(uin + rowp + xpair, vu[0], vu[1]);
            tb_ld_pair(bb + rowp + xpair, vb[0], vb[1]);
        } else {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                vu[c] = Tr<S>::ld(uin[rowp + xc[c]]);
                vb[c] = Tr<S>::ld(bb[rowp + xc[c]]);
            }
        }
    };

#pragma unroll
    for (int s = 0; s < D; ++s) load_row(r_first + dir * s, R.U[s], R.B[s]);

    // pipeline fill, unrolled: step i needs levels 1 .. i/2
#pragma unroll
    for (int i = 0; i < F; ++i) {
        const int s = i % D;
        const int lmax = min(T, i / 2);
        tb_step<S, T, C, D, FILL, HINT>(R, s, lmax, r_first + dir * i, cf, upd, ny, Tact, y0, y1, rowbytes, lanebase, rs,
                                  dir);
        load_row(r_first + dir * (i + D), R.U[s], R.B[s]);
        // keep each row load in its step: bunched at the end of the loop body they would be
        // waited for at the top of the next iteration
        __builtin_amdgcn_sched_barrier(0);
    }
    // steady state: all levels.  Binary64 at 10 levels (WIDE) runs K = lcm(D, 2) steps per
    // iteration, so that the load slots and the two-row window rotate by renaming (b's delay
    // line still needs copies at the back edge), then D steps per iteration for the rest;
    // the other cases run D steps per iteration, which measured faster for them.  The last
    // iteration may run past rl: its rows are loaded clamped and never stored.
    constexpr int K = (WIDE && sizeof(S) == 8 && T >= 10) ? tb_lcm(D, 2) : D;
    int i0 = F;
    if constexpr (K != D) {
        for (; i0 + K <= nsteps; i0 += K) {
#pragma unroll
            for (int q = 0; q < K; ++q) {
                const int r = r_first + dir * (i0 + q);
                tb_step<S, T, C, D, STEADY, HINT>(R, q % D, T, r, cf, upd, ny, Tact, y0, y1, rowbytes, lanebase, rs,
                                            dir);
                load_row(r + dir * D, R.U[q % D], R.B[q % D]);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    for (; i0 < nsteps; i0 += D) {
#pragma unroll
        for (int s = 0; s < D; ++s) {
            const int r = r_first + dir * (i0 + s);
            tb_step<S, T, C, D, STEADY, HINT>(R, s, T, r, cf, upd, ny, Tact, y0, y1, rowbytes, lanebase, rs, dir);
            load_row(r + dir * D, R.U[s], R.B[s]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// EDGES: whether tiles on the grid's edges get their own variants (fill checked, steady
// state checking columns only).  Each variant adds to the kernel's register count, which is
// the maximum over all of them; callers whose kernel is already near a waves-per-SIMD step
// use two variants only.  WIDE: whether binary64 at 10 levels may unroll its steady loop
// over lcm(D, 2) steps (the batch kernel, which also holds the residual path, may not: it
// would fall to one wave per SIMD).
template <class S, int T, int C, int D, bool EDGES = true, bool WIDE = true, int HINT = 0>
__device__ __forceinline__ void tb_tile(const S* __restrict__ uin, S* __restrict__ uout,
                                        const S* __restrict__ bb, int64_t px, int nx, int ny,
                                        const typename Tr<S>::C (&cf)[T], int Tact, int st, int sg, int H,
                                        int flip = 0)
{
    constexpr int SW = 64 * C - 2 * T;
    const int64_t xs = 1 + (int64_t)st * SW - T;
    const int y0 = 1 + sg * H;
    const int y1 = min(y0 + H, ny + 1);
    // computed rows are y0-T+1 .. y1+T-2, computed columns the strip's
    const bool top = y0 - T + 1 < 1;
    const bool bottom = y1 + T - 2 > ny;
    const bool cols = xs < 1 || xs + 64 * C - 1 > nx;
    // Segments of one parity stream upwards, so that the halo rows two neighbouring segments
    // share are read by both at the same time (both at their start or both at their end) and
    // the second read can come from L2; (S + N) equals (N + S) exactly, so the direction
    // changes no result.  flip swaps the parities: launched alternately, each launch starts
    // every segment on the rows the previous launch touched last, which the device's
    // memory-side cache is then most likely to still hold.  A tile that reaches the top ring
    // streams down and one that reaches the bottom ring streams up: its rows outside the grid
    // then all come in the pipeline fill, and only the fill checks rows.
    int dir = ((sg + flip) & 1) ? -1 : 1;
    if (top) dir = 1;
    if (bottom) dir = -1;
    if constexpr (!EDGES || (sizeof(S) == 8 && T < 10)) {
        // binary64 below 10 levels keeps two variants: more would raise the kernel's register
        // count past three waves per SIMD at 8 levels (at 10 it holds two waves either way)
        if (Tact < T || top || bottom || cols)
            tb_tile_body<S, T, C, D, TB_FULL, TB_FULL, WIDE, HINT>(uin, uout, bb, px, nx, ny, cf, Tact, st, sg, H, dir);
        else
            tb_tile_body<S, T, C, D, TB_CLEAN, TB_CLEAN, WIDE, HINT>(uin, uout, bb, px, nx, ny, cf, Tact, st, sg, H, dir);
        return;
    }
    if (Tact < T || (top && bottom)) {
        tb_tile_body<S, T, C, D, TB_FULL, TB_FULL, WIDE, HINT>(uin, uout, bb, px, nx, ny, cf, Tact, st, sg, H, dir);
    } else if (top || bottom) {
        if (cols)
            tb_tile_body<S, T, C, D, TB_FULL, TB_COLS, WIDE, HINT>(uin, uout, bb, px, nx, ny, cf, Tact, st, sg, H, dir);
        else
            tb_tile_body<S, T, C, D, TB_FULL, TB_CLEAN, WIDE, HINT>(uin, uout, bb, px, nx, ny, cf, Tact, st, sg, H, dir);
    } else if (cols) {
        tb_tile_body<S, T, C, D, TB_COLS, TB_COLS, WIDE, HINT>(uin, uout, bb, px, nx, ny, cf, Tact, st, sg, H, dir);
    } else {
        tb_tile_body<S, T, C, D, TB_CLEAN, TB_CLEAN, WIDE, HINT>(uin, uout, bb, px, nx, ny, cf, Tact, st, sg, H, dir);
    }
}

}  // namespace srj
