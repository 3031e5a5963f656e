// Temporally blocked 3D SRJ sweep for gfx950 (CDNA4, wave64).
//
// T consecutive scheduled sweeps (Sec. 2; each step the 7-point form of Sec. 3.1's update
// with d = 3, evaluated with the association and rounding of the unfused kernel, so the
// result is bit-identical to T unfused sweeps) are applied in one launch.  A block of NW waves
// (16, or 15 where that fills more compute units) owns an x-y tile of 64 columns (one per
// lane) by 2 NW rows (2 per wave) and streams a run of z planes through it.  At step k the block takes plane k (level 0) and computes level l for
// plane k - l, l = 1..T, from level l-1 planes k-l-1, k-l and k-l+1: each lane keeps, per
// level, the two older planes of its 2 points in registers; x neighbours cross lanes by DPP
// shifts, y neighbours are the lane's own rows except across wave boundaries, where the
// boundary rows of each level are exchanged through LDS (double-buffered by step parity, one
// barrier per step).  One HBM read of u and b and one write of u serve T sweeps; tiles overlap
// by T columns and rows on each side and z runs by T planes, the overlap being recomputed.
// Binary64 stores carry the non-temporal hint (kTbStoreNt).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>

#include "formats.h"
#include "kernels.h"
#include "tb_core.h"

namespace srj {

constexpr int k3_lcm(int a, int b)
{
    int x = a, y = b;
    while (y) {
        const int t = x % y;
        x = y;
        y = t;
    }
    return a / x * b;
}

template <int T> struct Coefs3T {
    double c[T];
};

constexpr int k3Rows = 2;  // rows per wave; a block of NW waves covers NW * k3Rows tile rows

template <class S, int T, int D, int NW>
__global__ __launch_bounds__(64 * NW) void k_sweep3d_tb(const S* __restrict__ uin, S* __restrict__ uout,
                                                    const S* __restrict__ bb, int64_t px, int64_t py, int nx,
                                                    int ny, int nz, Coefs3T<T> co, int Tact, int ntx, int nty,
                                                    int ntz, int zs, int dir)
{
    using Cm = typename Tr<S>::C;
    constexpr int SX = 64 - 2 * T;        // output columns per tile
    constexpr int SY = (NW * k3Rows) - 2 * T;   // output rows per tile
    __shared__ Cm xch[2][T][NW][2][64];

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // consecutive block indices go to different XCDs; remap them so that each XCD works a
    // contiguous band of tiles and neighbouring tiles share their halo reads in one L2
    const int nblk = (int)gridDim.x;  // a multiple of 8 (padded by the launcher)
    const int bid = (int)(blockIdx.x & 7) * (nblk >> 3) + (int)(blockIdx.x >> 3);
    if (bid >= ntx * nty * ntz) return;  // padding block: the whole block leaves
    const int tx = bid % ntx, ty = (bid / ntx) % nty, tz = bid / (ntx * nty);
    const int64_t pl = px * py;

    const int x = 1 + tx * SX - T + lane;
    const int64_t xcl = x < 0 ? 0 : (x > nx + 1 ? nx + 1 : x);
    const bool updx = x >= 1 && x <= nx;
    const bool outx = updx && lane >= T && lane < 64 - T;
    int yr[k3Rows];
    bool updy[k3Rows], outy[k3Rows];
    int64_t colp[k3Rows];
#pragma unroll
    for (int r = 0; r < k3Rows; ++r) {
        const int trow = w * k3Rows + r;
        yr[r] = 1 + ty * SY - T + trow;
        updy[r] = yr[r] >= 1 && yr[r] <= ny;
        outy[r] = updy[r] && trow >= T && trow < (NW * k3Rows) - T;
        const int64_t yc = yr[r] < 0 ? 0 : (yr[r] > ny + 1 ? ny + 1 : yr[r]);
        colp[r] = yc * px + xcl;
    }
    const int z0 = 1 + tz * zs;
    const int z1 = min(z0 + zs, nz + 1);
    const int kb = z0 - T;
    const int ke = z1 - 1 + T;
    // dir = +1 streams the run's planes upwards (level l works on plane k - l), -1 downwards
    // (plane k + l); the z pair of the sum is then formed as (U + D), the same IEEE sum as
    // (D + U).  Launches alternate it, so that each starts on the planes the previous one
    // touched last.
    const int kfirst = dir > 0 ? kb : ke;
    const int nsteps = ke - kb + 1;

    Cm cf[T];
#pragma unroll
    for (int l = 0; l < T; ++l) cf[l] = (Cm)co.c[l];

    // stores go through a buffer resource over the output plane whose range check drops
    // masked lanes (offset pushed below zero), rows (offset pushed past the record count) and
    // planes outside the run (record count 0)
    const int plbytes = (int)(pl * (int64_t)sizeof(S));
    const int lanebase = outx ? x * (int)sizeof(S) : INT_MIN;

    Cm w1[T][k3Rows], w2[T][k3Rows], bq[T][k3Rows];
#pragma unroll
    for (int l = 0; l < T; ++l)
#pragma unroll
        for (int r = 0; r < k3Rows; ++r) w1[l][r] = w2[l][r] = bq[l][r] = (Cm)0;

    auto load_plane = [&](int k, Cm* vu, Cm* vb) {
        const int64_t zp = (int64_t)max(0, min(k, nz + 1)) * pl;
#pragma unroll
        for (int r = 0; r < k3Rows; ++r) {
            vu[r] = Tr<S>::ld(uin[zp + colp[r]]);
            vb[r] = Tr<S>::ld(bb[zp + colp[r]]);
        }
    };

    Cm U[D][k3Rows], B[D][k3Rows];
#pragma unroll
    for (int s = 0; s < D; ++s) load_plane(kfirst + dir * s, U[s], B[s]);

    const int wu = max(w - 1, 0), wd = min(w + 1, NW - 1);
    // K steps per loop iteration, K a multiple of D (the load slots), 2 (the two older planes
    // per level) and T (the delay line of b): every register then plays the same role at both
    // ends of the loop body and the back edge needs no copies.  The last iteration may run up
    // to K - 1 planes past the run's last step: they are loaded clamped and never stored.
    constexpr int K = k3_lcm(k3_lcm(D, 2), T);
    for (int i0 = 0; i0 < nsteps; i0 += K) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const int s = q % D;
            const int k = kfirst + dir * (i0 + q);
            const int cur = k & 1, prev = cur ^ 1;
            Cm in[k3Rows];
#pragma unroll
            for (int r = 0; r < k3Rows; ++r) in[r] = U[s][r];
            xch[cur][0][w][0][lane] = in[0];
            xch[cur][0][w][1][lane] = in[k3Rows - 1];
#pragma unroll
            for (int l = 1; l <= T; ++l) {
                // level l on plane p = k - dir l; its y neighbours across wave boundaries are
                // the neighbouring waves' rows of plane p at level l-1, published in the
                // previous step
                const Cm up = xch[prev][l - 1][wu][1][lane];
                const Cm dn = xch[prev][l - 1][wd][0][lane];
                const int p = k - dir * l;
                const bool pok = (p >= 1) & (p <= nz) & (l <= Tact);
                Cm out[k3Rows], vs[k3Rows];
#pragma unroll
                for (int r = 0; r < k3Rows; ++r) {
                    const Cm m = w1[l - 1][r];
                    const Cm W = dpp_from_left(m);
                    const Cm E = dpp_from_right(m);
                    const Cm Sn = (r == 0) ? up : w1[l - 1][r - 1];
                    const Cm Nn = (r == k3Rows - 1) ? dn : w1[l - 1][r + 1];
                    const Cm sm = ((W + E) + (Sn + Nn)) + (w2[l - 1][r] + in[r]);
                    const Cm t = (sm + bq[l - 1][r]) - (Cm)6 * m;
                    vs[r] = m + cf[l - 1] * t;
                }
                tb_round<S>(vs);
#pragma unroll
                for (int r = 0; r < k3Rows; ++r) {
                    Cm v = vs[r];
                    asm("" : "+v"(v));
                    out[r] = (pok && updx && updy[r]) ? v : w1[l - 1][r];
                }
#pragma unroll
                for (int r = 0; r < k3Rows; ++r) {
                    w2[l - 1][r] = w1[l - 1][r];
                    w1[l - 1][r] = in[r];
                    in[r] = out[r];
                }
                if (l < T) {
                    xch[cur][l][w][0][lane] = in[0];
                    xch[cur][l][w][1][lane] = in[k3Rows - 1];
                }
            }
            // level T of plane k - dir T
            const int pT = k - dir * T;
            const bool zout = (pT >= z0) & (pT < z1);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(uout + (int64_t)min(max(pT, 0), nz + 1) * pl), (short)0, zout ? plbytes : 0, 0x00020000);
#pragma unroll
            for (int r = 0; r < k3Rows; ++r) {
                const int rowpart = outy[r] ? (int)((int64_t)yr[r] * px * (int64_t)sizeof(S)) : kTbMasked;
                tb_store<sizeof(S) == 8 ? kTbStoreNt : 0>(Tr<S>::st(in[r]), rs, rowpart + lanebase);
            }
#pragma unroll
            for (int l = T - 1; l > 0; --l)
#pragma unroll
                for (int r = 0; r < k3Rows; ++r) bq[l][r] = bq[l - 1][r];
#pragma unroll
            for (int r = 0; r < k3Rows; ++r) bq[0][r] = B[s][r];
            __syncthreads();
            load_plane(k + dir * D, U[s], B[s]);
        }
    }
}

template <class S, int T, int D, int NW>
static int tb3_resident_blocks()
{
    static const int blocks = [] {
        int nb = 0, dev = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep3d_tb<S, T, D, NW>, 64 * NW, 0) != hipSuccess)
            nb = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 1;
        return std::max(1, nb) * std::max(1, ncu);
    }();
    return blocks;
}

// Launch shape of depth T with NW-wave blocks: tiles per axis and z runs of zs planes, as
// many runs as fill the resident block slots once (at least one), balanced.
struct Tb3Shape {
    int ntx, nty, ntz, zs;
};
template <class S, int T, int D, int NW>
static Tb3Shape tb3_shape(const Geo& g)
{
    constexpr int SX = 64 - 2 * T, SY = NW * k3Rows - 2 * T;
    Tb3Shape sh;
    sh.ntx = (int)((g.nx + SX - 1) / SX);
    sh.nty = (int)((g.ny + SY - 1) / SY);
    int ntz = std::max(1, tb3_resident_blocks<S, T, D, NW>() / (sh.ntx * sh.nty));
    int zs = (int)((g.nz + ntz - 1) / ntz);
    zs = std::max(1, std::min(zs, (int)g.nz));
    ntz = (int)((g.nz + zs - 1) / zs);
    sh.ntz = ntz;
    sh.zs = (int)((g.nz + ntz - 1) / ntz);
    return sh;
}

template <class S, int T, int D, int NW>
static void tb3d_launch(const S* in, S* out, const S* b, const Geo& g, const Coefs3T<T>& ct, int Tact, int dir,
                        hipStream_t s)
{
    const Tb3Shape sh = tb3_shape<S, T, D, NW>(g);
    const int nblk = (sh.ntx * sh.nty * sh.ntz + 7) / 8 * 8;
    hipLaunchKernelGGL((k_sweep3d_tb<S, T, D, NW>), dim3(nblk), dim3(64 * NW), 0, s, in, out, b, g.px, g.py, (int)g.nx,
                       (int)g.ny, (int)g.nz, ct, Tact, sh.ntx, sh.nty, sh.ntz, sh.zs, dir);
}

// Tiles of 16 waves (32 rows) by default; 15 waves (30 rows) when that fills more of the
// resident block slots in one round without needing a second (512^2 planes at T = 4: 240
// tiles instead of 220 for 256 compute units), each tile then doing 6% less work.
template <class S, int T, int D>
static bool tb3_use15(const Geo& g)
{
    auto tiles = [&](int nw) {
        const int64_t SX = 64 - 2 * T, SY = nw * k3Rows - 2 * T;
        return ((g.nx + SX - 1) / SX) * ((g.ny + SY - 1) / SY);
    };
    const int64_t t16 = tiles(16), t15 = tiles(15);
    const int64_t slots = tb3_resident_blocks<S, T, D, 16>();
    return t16 < slots && t15 > t16 && t15 <= slots && 15 * k3Rows > 2 * T + 8;
}

template <class S, int T, int D>
static void tb3d(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int Tact, int dir, hipStream_t s)
{
    Coefs3T<T> ct;
    for (int l = 0; l < T; ++l) ct.c[l] = l < Tact ? co.c[l] : 0.0;
    if (tb3_use15<S, T, D>(g))
        tb3d_launch<S, T, D, 15>(in, out, b, g, ct, Tact, dir, s);
    else
        tb3d_launch<S, T, D, 16>(in, out, b, g, ct, Tact, dir, s);
}

// Modelled time per sweep of depth T, in units of the per-step cost: rounds of blocks x the
// steps one block streams (its z run plus 2T, rounded up to the unrolled loop's K steps) x a
// per-step cost a + b T, over the T sweeps a launch advances.  a = 1.04 and b = 0.154 (us)
// were fitted to the binary64 launches at 512^3 (4 and 5 sweeps); the model then picks the
// measured fastest depth at 256^3, 384^3 (where 5 gives 160 blocks for 256 compute units),
// 512^3 and 640^3.
template <class S, int T, int D, int NW>
static double tb3_cost_nw(const Geo& g)
{
    const Tb3Shape sh = tb3_shape<S, T, D, NW>(g);
    const int64_t slots = std::max(1, tb3_resident_blocks<S, T, D, NW>());
    const int64_t blocks = (int64_t)sh.ntx * sh.nty * sh.ntz;
    const int64_t rounds = (blocks + slots - 1) / slots;
    constexpr int K = k3_lcm(k3_lcm(D, 2), T);
    const int64_t steps = (sh.zs + 2 * T + K - 1) / K * K;
    return (double)rounds * (double)steps * (1.04 + 0.154 * T) / T;
}

template <class S, int T, int D>
static double tb3_cost(const Geo& g)
{
    return tb3_use15<S, T, D>(g) ? tb3_cost_nw<S, T, D, 15>(g) : tb3_cost_nw<S, T, D, 16>(g);
}

// Depth 5, 4 or 3, whichever the model gives the lowest time per sweep (ties to the deeper).
template <class S, int D>
static int tb3_pick(const Geo& g)
{
    int best = 5;
    double c = tb3_cost<S, 5, D>(g);
    const double c4 = tb3_cost<S, 4, D>(g), c3 = tb3_cost<S, 3, D>(g);
    if (c4 < c) {
        best = 4;
        c = c4;
    }
    if (c3 < c) best = 3;
    return best;
}

template <class S, int D>
static void tb3d_TD(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int T, int dir, hipStream_t s)
{
    switch (T) {
    case 1: tb3d<S, 1, D>(in, out, b, g, co, 1, dir, s); break;
    case 2: tb3d<S, 2, D>(in, out, b, g, co, 2, dir, s); break;
    case 3: tb3d<S, 3, D>(in, out, b, g, co, 3, dir, s); break;
    case 4: tb3d<S, 4, D>(in, out, b, g, co, 4, dir, s); break;
    default: tb3d<S, 5, D>(in, out, b, g, co, 5, dir, s); break;
    }
}

// Planes in flight per wave: 3 in binary64 (at 5 sweeps per launch 4% faster than 2, though
// it spills 8 VGPRs; 4 was 17% slower), 2 in the 4- and 2-byte formats (3 was 4-9% slower).
template <class S>
static void tb3d_T(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int T, int dir, hipStream_t s)
{
    if constexpr (sizeof(S) == 8)
        tb3d_TD<S, 3>(in, out, b, g, co, T, dir, s);
    else
        tb3d_TD<S, 2>(in, out, b, g, co, T, dir, s);
}

int fused3d_default_depth(const Geo& g, Fmt f)
{
    if (g.ndim != 3) return 0;
    switch (f) {
    case FMT_F64: return tb3_pick<double, 3>(g);
    case FMT_F32: return tb3_pick<float, 2>(g);
    default: return tb3_pick<bf16_t, 2>(g);
    }
}

hipError_t launch_sweep_fused3d(Fmt f, const void* in, void* out, const void* b, const Geo& g,
                                const Coefs& co, int T, int flip, hipStream_t s)
{
    if (g.ndim != 3 || T < 1 || T > kMaxFuse3d) return hipErrorInvalidValue;
    const int dir = (flip & 1) ? -1 : 1;
    SRJ_DISPATCH(f, tb3d_T<S>((const S*)in, (S*)out, (const S*)b, g, co, T, dir, s));
    return hipGetLastError();
}

}  // namespace srj
