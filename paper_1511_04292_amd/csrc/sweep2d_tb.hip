// Temporally blocked 2D SRJ sweep for gfx950 (CDNA4, wave64).
//
// T consecutive scheduled sweeps (Sec. 2; each step as in Sec. 3.1, Eq. 2nd-order_CD,
// evaluated with the association and rounding of the unfused kernel, so the result is
// bit-identical to T unfused sweeps) are applied in one launch.  Each wavefront owns a
// strip of 64*C columns (C per lane) and a segment of rows, streams the rows (downwards or
// upwards: neighbouring segments alternate, and every launch flips them) and keeps T time
// levels of a 3-row window in registers: one HBM read of u and b and one write of u serve T
// sweeps.  Horizontal neighbours cross lanes by DPP lane shifts; no LDS and no barriers are
// needed because every wave is independent (strips overlap by T columns on each side,
// segments by T rows, the overlap being recomputed).  The last template argument is the
// stores' cache hint (kTbStoreNt or 0), chosen per plan for binary64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "formats.h"
#include "kernels.h"
#include "tb_core.h"

namespace srj {

// --------------------------------------------------- temporally blocked 2D sweeps

template <int T> struct CoefsT {
    double c[T];
};

// Blocks are remapped so that each of the 8 XCDs works on a contiguous band of tiles,
// keeping the overlapping halo reads of neighbouring waves in one L2.
// The 4- and 2-byte formats are held to 3 waves per SIMD (168 VGPRs): at 10 levels the
// compiler would otherwise take 185 and leave 2; binary64 is left to the compiler.
template <class S, int T, int C, int D, int HINT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 1 : 3)))
void k_sweep2d_tb(const S* __restrict__ uin, S* __restrict__ uout, const S* __restrict__ bb, int64_t px, int nx,
                  int ny, CoefsT<T> co, int nstrip, int nwaves, int H, int flip)
{
    using Cm = typename Tr<S>::C;
    const int nblk = (int)gridDim.x;  // a multiple of 8 (padded by the launcher)
    const int blk = (int)(blockIdx.x & 7) * (nblk >> 3) + (int)(blockIdx.x >> 3);
    // the wave index is uniform across the wave: keep it (and all loop bounds) in SGPRs
    const int wid = __builtin_amdgcn_readfirstlane(blk * 4 + (int)(threadIdx.x >> 6));
    if (wid >= nwaves) return;
    Cm cf[T];
#pragma unroll
    for (int l = 0; l < T; ++l) cf[l] = (Cm)co.c[l];
    tb_tile<S, T, C, D, true, true, HINT>(uin, uout, bb, px, nx, ny, cf, T, wid % nstrip, wid / nstrip, H, flip);
}

// Waves of one kernel instance that the device holds at once: blocks per CU (from the
// kernel's register and LDS use) x 4 waves x CUs.
template <class S, int T, int C, int D, int HINT>
static int tb_resident_waves()
{
    static const int waves = [] {
        int nb = 0, dev = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_sweep2d_tb<S, T, C, D, HINT>, 256, 0) != hipSuccess)
            nb = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            ncu = 1;
        return std::max(1, nb) * 4 * std::max(1, ncu);
    }();
    return waves;
}

template <class S, int T, int C, int D, int HINT>
static void tb2d(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int H, int flip,
                 hipStream_t s)
{
    constexpr int SW = 64 * C - 2 * T;
    CoefsT<T> ct;
    for (int l = 0; l < T; ++l) ct.c[l] = co.c[l];
    const int nstrip = (int)((g.nx + SW - 1) / SW);
    if (H <= 0) {
        // One round: as many row segments as leave every resident wave slot one tile, so
        // that all waves start together and the device stays full until they end.  Below
        // 2T rows a tile would spend most of its steps filling the pipeline.
        const int per_strip = std::max(1, tb_resident_waves<S, T, C, D, HINT>() / nstrip);
        H = std::max((int)((g.ny + per_strip - 1) / per_strip), std::max(2 * T, 8));
    }
    H = std::min(H, tb_max_rows(g.px, (int)sizeof(S)));
    const int nseg = (int)((g.ny + H - 1) / H);
    const int nwaves = nstrip * nseg;
    const int nblk = ((nwaves + 3) / 4 + 7) / 8 * 8;
    hipLaunchKernelGGL((k_sweep2d_tb<S, T, C, D, HINT>), dim3(nblk), dim3(256), 0, s, in, out, b, g.px,
                       (int)g.nx, (int)g.ny, ct, nstrip, nwaves, H, flip);
}

// The non-temporal store hint applies to binary64 only (see kTbStoreNt).
template <class S, int T, int C, int D>
static void tb2d_h(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int H, int flip, bool nt,
                   hipStream_t s)
{
    if constexpr (sizeof(S) == 8) {
        if (nt) {
            tb2d<S, T, C, D, kTbStoreNt>(in, out, b, g, co, H, flip, s);
            return;
        }
    }
    tb2d<S, T, C, D, 0>(in, out, b, g, co, H, flip, s);
}

template <class S, int C, int D>
static void tb2d_T(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int T, int H, int flip, bool nt,
                   hipStream_t s)
{
    switch (T) {
    case 1: tb2d_h<S, 1, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    case 2: tb2d_h<S, 2, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    case 3: tb2d_h<S, 3, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    case 4: tb2d_h<S, 4, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    case 5: tb2d_h<S, 5, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    case 6: tb2d_h<S, 6, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    case 7: tb2d_h<S, 7, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    case 8: tb2d_h<S, 8, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    case 9: tb2d_h<S, 9, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    default: tb2d_h<S, 10, C, D>(in, out, b, g, co, H, flip, nt, s); break;
    }
}

// Rows in flight per wave: 3 for binary64 (its unrolled loop then matches the 3-row window
// and the kernel keeps 3 waves per SIMD at 8 sweeps), 4 for the 4-byte and 2-byte formats.
template <class S>
static void tb2d_dispatch(const S* in, S* out, const S* b, const Geo& g, const Coefs& co, int T,
                          int H, int flip, bool nt, hipStream_t s)
{
    constexpr int C = 2;
    if constexpr (sizeof(S) == 8)
        tb2d_T<S, C, 3>(in, out, b, g, co, T, H, flip, nt, s);
    else
        tb2d_T<S, C, 4>(in, out, b, g, co, T, H, flip, false, s);
}

hipError_t launch_sweep_fused(Fmt f, const void* in, void* out, const void* b, const Geo& g,
                              const Coefs& co, int T, int H, int flip, bool nt, hipStream_t s)
{
    if (g.ndim != 2 || T < 1 || T > kMaxFuse || H < 0) return hipErrorInvalidValue;  // H = 0: automatic
    flip &= 1;
    SRJ_DISPATCH(f, tb2d_dispatch<S>((const S*)in, (S*)out, (const S*)b, g, co, T, H, flip, nt, s));
    return hipGetLastError();
}


}  // namespace srj
