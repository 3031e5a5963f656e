// Batched SRJ solves on gfx950: many independent 2D grids of different sizes, each with its
// own schedule (Sec. 2), solved to a relative residual by FP64 iterative refinement around
// SRJ sweeps in the batch's storage format.
//
// Every problem carries its state on the device (BState); one iteration of the batch is two
// launches over fixed work lists that cover all problems:
//   * k_batch_sweep: every wave takes tiles of problems that are sweeping and applies up to
//     T scheduled sweeps to the correction d (the register-pipelined tile of tb_core.h);
//     the wave that finishes a problem's last tile advances that problem's sweep counter
//     and, at the end of its inner solve, hands it to the residual step;
//   * k_batch_residual: every block takes 8 rows of problems awaiting a residual, forms
//     u' = u + d, r = b - A u' (binary64), the cast right-hand side for the next inner
//     solve and a zero start for it, and writes its partial sums; the block that finishes
//     a problem's last rows reduces them in a fixed order and decides: converged, diverged,
//     out of outer steps, or sweep again.
// No kernel waits on another block: completion is counted with atomics and the last
// arrival acts, so every wave always runs to its end.  The host replays a graph of such
// iterations until no problem remains.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "batch.h"
#include "formats.h"
#include "tb_core.h"

namespace srj {

constexpr int kBatchT = 8;  // sweeps fused per batch sweep launch
constexpr int kBatchRows = 8;

int batch_fuse() { return kBatchT; }

// largest j in [0, count) with prefix[j] <= item (prefix[count] = total)
__device__ __forceinline__ int find_problem(const int* __restrict__ prefix, int count, int item)
{
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ void k_batch_start(uint64_t* t0)
{
    if (threadIdx.x == 0) *t0 = wall_clock64();
}

template <class S, int T, int C, int D>
__global__ __launch_bounds__(256) void k_batch_sweep(const BProb* __restrict__ probs, BState* st,
                                                     const int* __restrict__ item_prefix,
                                                     const double* __restrict__ coef, BRun run)
{
    using Cm = typename Tr<S>::C;
    const int lane = threadIdx.x & 63;
    const int nslots = (int)gridDim.x * 4;
    const int slot = __builtin_amdgcn_readfirstlane((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6));
    for (int item = slot; item < run.nitems; item += nslots) {
        const int j = find_problem(item_prefix, run.count, item);
        const BProb& P = probs[j];
        if (st[j].phase != BP_SWEEP) continue;
        const int k = st[j].k;
        const int dcur = st[j].dcur;
        const int Tj = min(T, P.inner_total - k);
        Cm cf[T];
#pragma unroll
        for (int l = 0; l < T; ++l) cf[l] = (l < Tj) ? (Cm)coef[P.coff + (k + l) % P.M] : (Cm)0;
        const int local = item - P.item0;
        tb_tile<S, T, C, D>((const S*)P.d[dcur], (S*)P.d[1 - dcur], (const S*)P.rlo, P.px, P.nx, P.ny, cf,
                            Tj, local % P.nstrip, local / P.nstrip, run.H);
        __threadfence();
        int old = 0;
        if (lane == 0) old = atomicAdd(&st[j].cnt_s, 1);
        old = __shfl(old, 0, 64);
        if (old == P.nitems - 1 && lane == 0) {
            __threadfence();
            const int nk = k + Tj;
            st[j].k = nk;
            st[j].dcur = 1 - dcur;
            st[j].cnt_s = 0;
            if (nk >= P.inner_total) st[j].phase = BP_RESIDUAL;
        }
    }
}

static __device__ __forceinline__ void bnanmax(double& m, double a)
{
    if (a > m || a != a) m = a;
}

template <class S>
__global__ __launch_bounds__(256) void k_batch_residual(const BProb* __restrict__ probs, BState* st,
                                                        const int* __restrict__ rb_prefix,
                                                        double* partials, BRun run)
{
    __shared__ double ss[4], sm[4];
    for (int item = (int)blockIdx.x; item < run.nrb; item += (int)gridDim.x) {
        const int j = find_problem(rb_prefix, run.count, item);
        const BProb& P = probs[j];
        if (st[j].phase != BP_RESIDUAL) continue;
        const int ucur = st[j].ucur, dcur = st[j].dcur;
        const double* __restrict__ u = P.u64[ucur];
        double* __restrict__ un = P.u64[1 - ucur];
        const S* __restrict__ d = (const S*)P.d[dcur];
        S* __restrict__ dz = (S*)P.d[1 - dcur];
        S* __restrict__ rl = (S*)P.rlo;
        const int64_t px = P.px;
        const int rb = item - P.rb0;
        double s = 0.0, m = 0.0;
        const int i1 = min(rb * kBatchRows + kBatchRows, P.ny);
        for (int i = rb * kBatchRows + 1; i <= i1; ++i) {
            for (int x = (int)threadIdx.x + 1; x <= P.nx; x += 256) {
                const int64_t p = (int64_t)i * px + x;
                // the refined iterate u + d, formed identically at the point and its neighbours
                const double c = u[p] + (double)Tr<S>::ld(d[p]);
                const double w = u[p - 1] + (double)Tr<S>::ld(d[p - 1]);
                const double e = u[p + 1] + (double)Tr<S>::ld(d[p + 1]);
                const double so = u[p - px] + (double)Tr<S>::ld(d[p - px]);
                const double no = u[p + px] + (double)Tr<S>::ld(d[p + px]);
                const double sn = (w + e) + (so + no);
                const double r = (sn + P.b64[p]) - 4.0 * c;
                un[p] = c;
                rl[p] = Tr<S>::from64(r);
                dz[p] = zero_of<S>();
                s = s + r * r;
                bnanmax(m, fabs(r));
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double so = __shfl_xor(s, o, 64);
            const double mo = __shfl_xor(m, o, 64);
            s = s + so;
            bnanmax(m, mo);
        }
        const int wv = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            ss[wv] = s;
            sm[wv] = m;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s = (ss[0] + ss[1]) + (ss[2] + ss[3]);
            m = sm[0];
            bnanmax(m, sm[1]);
            bnanmax(m, sm[2]);
            bnanmax(m, sm[3]);
            partials[2 * (P.pbase + rb)] = s;
            partials[2 * (P.pbase + rb) + 1] = m;
            __threadfence();
            const int old = atomicAdd(&st[j].cnt_r, 1);
            if (old == P.nrb - 1) {
                __threadfence();
                double tot = 0.0;
                for (int b = 0; b < P.nrb; ++b)
                    tot = tot + __hip_atomic_load(&partials[2 * (P.pbase + b)], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
                const double rr = sqrt(tot) / sqrt(*P.bt2);
                int outer = st[j].outer;
                int ph;
                if (!(rr == rr) || rr > 1.7976931348623157e308) {
                    ph = BP_DIVERGED;
                } else if (rr <= run.tol) {
                    ph = BP_DONE;
                } else if (outer >= run.max_outer) {
                    ph = BP_NOCONV;
                } else {
                    ph = BP_SWEEP;
                    outer += 1;
                }
                st[j].relres = rr;
                st[j].ucur = 1 - ucur;
                st[j].dcur = 1 - dcur;
                st[j].k = 0;
                st[j].outer = outer;
                st[j].cnt_r = 0;
                if (ph == BP_DONE) st[j].t_end = wall_clock64();
                st[j].phase = ph;
                if (ph != BP_SWEEP) atomicSub(run.remaining, 1);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_batch_start(uint64_t* t0, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_start, dim3(1), dim3(64), 0, s, t0);
    return hipGetLastError();
}

hipError_t launch_batch_sweep(Fmt f, const BProb* probs, BState* st, const int* item_prefix,
                              const double* coef, const BRun& run, int grid_blocks, hipStream_t s)
{
    constexpr int C = 2, D = 4;
    switch (f) {
    case FMT_F64:
        hipLaunchKernelGGL((k_batch_sweep<double, kBatchT, C, D>), dim3(grid_blocks), dim3(256), 0, s, probs, st,
                           item_prefix, coef, run);
        break;
    case FMT_F32:
        hipLaunchKernelGGL((k_batch_sweep<float, kBatchT, C, D>), dim3(grid_blocks), dim3(256), 0, s, probs, st,
                           item_prefix, coef, run);
        break;
    default:
        hipLaunchKernelGGL((k_batch_sweep<bf16_t, kBatchT, C, D>), dim3(grid_blocks), dim3(256), 0, s, probs, st,
                           item_prefix, coef, run);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_batch_residual(Fmt f, const BProb* probs, BState* st, const int* rb_prefix,
                                 double* partials, const BRun& run, int grid_blocks, hipStream_t s)
{
    SRJ_DISPATCH(f, hipLaunchKernelGGL(k_batch_residual<S>, dim3(grid_blocks), dim3(256), 0, s, probs, st,
                                       rb_prefix, partials, run));
    return hipGetLastError();
}

}  // namespace srj
