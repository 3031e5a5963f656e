// Batched SRJ solves on gfx950: many independent 2D grids of different sizes, each with its
// own schedule (Sec. 2), solved to a relative residual by FP64 iterative refinement around
// SRJ sweeps in the batch's storage format.
//
// Every problem carries its state on the device (BState) and is cut into tiles (column strip
// x row segment).  One iteration of the batch is one launch over the work list of the tiles
// of all running problems; a wave that takes a tile looks at its problem's phase and
//   * SWEEP: applies up to T scheduled sweeps to the correction d on the tile (the
//     register-pipelined tile of tb_core.h);
//   * RESIDUAL: forms, on the tile's output points, u' = u + d, r = b - A u' (binary64), the
//     cast right-hand side of the next inner solve and a zero start for it, and writes the
//     tile's partial sums.
// The wave that finishes the last tile of a problem in a launch advances that problem: after
// sweeps it moves the sweep counter (and hands the problem to the residual at the end of an
// inner solve); after a residual it reduces the tile sums in a fixed order and decides:
// converged, diverged, out of outer steps, or sweep again.  No wave waits on another:
// completion is counted with an atomic and the last arrival acts, so every wave always runs
// to its end.  The host replays a graph of such launches until no problem remains.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch.h"
#include "formats.h"
#include "tb_core.h"

namespace srj {

constexpr int kBatchT = 10; // sweeps fused per launch
constexpr int kBatchC = 2;  // columns per lane
constexpr int kBatchD = 3;  // rows in flight per wave (the kernel then keeps 3 waves per SIMD
                             // with the edge-tile variants)

int batch_fuse() { return kBatchT; }

__global__ void k_batch_start(uint64_t* t0)
{
    if (threadIdx.x == 0) *t0 = wall_clock64();
}

static __device__ __forceinline__ void bnanmax(double& m, double a)
{
    if (a > m || a != a) m = a;
}

// Residual on the output points of tile (strip st, segment sg): the same points the sweep
// tile stores, so the tiles of a problem cover its interior once.  Returns the lane's sum
// of r^2 and max |r|.
template <class S, int T, int C>
__device__ __forceinline__ void residual_tile(const BProb& P, int ucur, int dcur, int st, int sg, double& s,
                                              double& m)
{
    constexpr int SW = 64 * C - 2 * T;
    const int lane = threadIdx.x & 63;
    const double* __restrict__ u = P.u64[ucur];
    double* __restrict__ un = P.u64[1 - ucur];
    const S* __restrict__ d = (const S*)P.d[dcur];
    S* __restrict__ dz = (S*)P.d[1 - dcur];
    S* __restrict__ rl = (S*)P.rlo;
    const int64_t px = P.px;
    const int64_t x0 = 1 + (int64_t)st * SW - T + (int64_t)lane * C;
    const int y0 = 1 + sg * P.H;
    const int y1 = min(y0 + P.H, P.ny + 1);
    bool on[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int off = lane * C + c;
        on[c] = off >= T && off < 64 * C - T && x0 + c >= 1 && x0 + c <= (int64_t)P.nx;
    }
    s = 0.0;
    m = 0.0;
    for (int i = y0; i < y1; ++i) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            if (!on[c]) continue;
            const int64_t p = (int64_t)i * px + x0 + c;
            // the refined iterate u + d, formed identically at the point and its neighbours
            const double ce = u[p] + (double)Tr<S>::ld(d[p]);
            const double w = u[p - 1] + (double)Tr<S>::ld(d[p - 1]);
            const double e = u[p + 1] + (double)Tr<S>::ld(d[p + 1]);
            const double so = u[p - px] + (double)Tr<S>::ld(d[p - px]);
            const double no = u[p + px] + (double)Tr<S>::ld(d[p + px]);
            const double sn = (w + e) + (so + no);
            const double r = (sn + P.b64[p]) - 4.0 * ce;
            un[p] = ce;
            rl[p] = Tr<S>::from64(r);
            dz[p] = zero_of<S>();
            s = s + r * r;
            bnanmax(m, fabs(r));
        }
    }
}

// As in the single-grid kernel, the 4- and 2-byte formats are held to 3 waves per SIMD.
template <class S, int T, int C, int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 8 ? 1 : 3)))
void k_batch_step(const BProb* __restrict__ probs, BState* st, BRun run)
{
    using Cm = typename Tr<S>::C;
    const int lane = threadIdx.x & 63;
    const int nslots = (int)gridDim.x * 4;
    const int slot = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
    const int n = __builtin_amdgcn_readfirstlane(*run.nitems);
    for (int it = slot; it < n; it += nslots) {
        const BItem e = run.items[it];
        const int j = __builtin_amdgcn_readfirstlane(e.prob);
        const int tile = __builtin_amdgcn_readfirstlane(e.tile);
        const BProb& P = probs[j];
        const int ph = __builtin_amdgcn_readfirstlane(st[j].phase);
        if (ph != BP_SWEEP && ph != BP_RESIDUAL) continue;
        const int k = __builtin_amdgcn_readfirstlane(st[j].k);
        const int ucur = __builtin_amdgcn_readfirstlane(st[j].ucur);
        const int dcur = __builtin_amdgcn_readfirstlane(st[j].dcur);
        const int nstrip = P.nstrip;
        const int sx = tile % nstrip, sg = tile / nstrip;
        int Tj = 0;
        if (ph == BP_SWEEP) {
            Tj = min(T, P.inner_total - k);
            Cm cf[T];
#pragma unroll
            for (int l = 0; l < T; ++l) cf[l] = (l < Tj) ? (Cm)run.coef[P.coff + (k + l) % P.M] : (Cm)0;
            // the stream direction alternates with the problem's launches, as in the
            // single-grid kernel
            tb_tile<S, T, C, D, true, false>((const S*)P.d[dcur], (S*)P.d[1 - dcur], (const S*)P.rlo, P.px, P.nx, P.ny, cf,
                                       Tj, sx, sg, P.H, (k / T) & 1);
        } else {
            double s, m;
            residual_tile<S, T, C>(P, ucur, dcur, sx, sg, s, m);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double so = __shfl_xor(s, o, 64);
                const double mo = __shfl_xor(m, o, 64);
                s = s + so;
                bnanmax(m, mo);
            }
            if (lane == 0) {
                run.partials[2 * (P.pbase + tile)] = s;
                run.partials[2 * (P.pbase + tile) + 1] = m;
            }
        }
        // A sweep tile's last arrival only moves the problem's counters, which are read in
        // later launches (kernel boundaries order them), so sweep tiles count without a fence:
        // an agent-scope fence writes back and invalidates the L2.  Residual tiles publish
        // their sums before counting, and the last one acquires them.
        if (ph == BP_RESIDUAL) __threadfence();
        int old = 0;
        if (lane == 0) old = atomicAdd(&st[j].cnt, 1);
        old = __shfl(old, 0, 64);
        if (old != P.ntiles - 1) continue;
        // last tile of problem j in this launch
        if (ph == BP_SWEEP) {
            if (lane == 0) {
                const int nk = k + Tj;
                st[j].k = nk;
                st[j].dcur = 1 - dcur;
                st[j].cnt = 0;
                if (nk >= P.inner_total) st[j].phase = BP_RESIDUAL;
            }
            continue;
        }
        __threadfence();
        // the whole wave reduces the tile sums: lane-strided partial sums, then a butterfly
        double tot = 0.0, mx = 0.0;
        for (int b = lane; b < P.ntiles; b += 64) {
            tot = tot + __hip_atomic_load(&run.partials[2 * (P.pbase + b)], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bnanmax(mx, __hip_atomic_load(&run.partials[2 * (P.pbase + b) + 1], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT));
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double so = __shfl_xor(tot, o, 64);
            const double mo = __shfl_xor(mx, o, 64);
            tot = tot + so;
            bnanmax(mx, mo);
        }
        if (lane == 0) {
            const double rr = sqrt(tot) / sqrt(*P.bt2);
            int outer = st[j].outer;
            int nph;
            if (!(rr == rr) || rr > 1.7976931348623157e308) {
                nph = BP_DIVERGED;
            } else if (rr <= run.tol) {
                nph = BP_DONE;
            } else if (outer >= run.max_outer) {
                nph = BP_NOCONV;
            } else {
                nph = BP_SWEEP;
                outer += 1;
            }
            st[j].relres = rr;
            st[j].ucur = 1 - ucur;
            st[j].dcur = 1 - dcur;
            st[j].k = 0;
            st[j].outer = outer;
            st[j].cnt = 0;
            if (nph == BP_DONE) st[j].t_end = wall_clock64();
            st[j].phase = nph;
            if (nph != BP_SWEEP) atomicSub(run.remaining, 1);
        }
    }
}

hipError_t launch_batch_start(uint64_t* t0, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_start, dim3(1), dim3(64), 0, s, t0);
    return hipGetLastError();
}

hipError_t launch_batch_step(Fmt f, const BProb* probs, BState* st, const BRun& run, int grid_blocks,
                             hipStream_t s)
{
    constexpr int T = kBatchT, C = kBatchC, D = kBatchD;
    switch (f) {
    case FMT_F64:
        hipLaunchKernelGGL((k_batch_step<double, T, C, D>), dim3(grid_blocks), dim3(256), 0, s, probs, st, run);
        break;
    case FMT_F32:
        hipLaunchKernelGGL((k_batch_step<float, T, C, D>), dim3(grid_blocks), dim3(256), 0, s, probs, st, run);
        break;
    default:
        hipLaunchKernelGGL((k_batch_step<bf16_t, T, C, D>), dim3(grid_blocks), dim3(256), 0, s, probs, st, run);
        break;
    }
    return hipGetLastError();
}

}  // namespace srj
