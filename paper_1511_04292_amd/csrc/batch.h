// Batched SRJ solves: many independent 2D grids, each with its own schedule, refined in
// FP64 around sweeps in the batch's storage format, advanced together by one kernel launch
// per iteration (see batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace srj {

// Immutable per-problem descriptor (device copy uploaded at solve start).
struct BProb {
    int32_t nx, ny;
    int64_t px;              // row pitch of every field of this problem (elements)
    double* u64[2];          // FP64 iterate ping-pong (origins, ring included)
    double* b64;             // FP64 scaled source h^2 f
    void* d[2];              // correction ping-pong in the sweep format
    void* rlo;               // residual cast to the sweep format (the inner right-hand side)
    const double* bt2;       // -> ||b~||^2 of this problem
    int32_t M, coff;         // cycle length and offset of its c_k in the coefficient table
    int32_t inner_total;     // sweeps per inner solve (inner_cycles * M)
    int32_t nstrip;          // column strips of a tile row
    int32_t ntiles;          // tiles (strips x row segments)
    int32_t H;               // output rows per tile
    int32_t pbase;           // first slot of its per-tile partial sums
    int32_t pad;
};

// Mutable per-problem state, written only by the kernels (single lane, vector stores).
enum { BP_SWEEP = 1, BP_DONE = 2, BP_DIVERGED = 3, BP_RESIDUAL = 4, BP_NOCONV = 5 };
struct BState {
    int32_t phase, k, ucur, dcur;
    int32_t outer, cnt, pad0, pad1;
    double relres;
    uint64_t t_end;
};

// One entry of the work list: a tile of a problem.
struct BItem {
    int32_t prob, tile;
};

// Per-solve constants and shared buffers.
struct BRun {
    double tol;
    int32_t max_outer;
    int32_t pad;
    const BItem* items;   // work list (tiles of the problems still running)
    const int* nitems;    // its length, rewritten by the host between graph replays
    const double* coef;   // c_k of every problem (BProb::coff)
    double* partials;     // per-tile residual partial sums (2 per tile)
    int* remaining;       // problems not yet finished
};

int batch_fuse();  // sweeps fused per launch

hipError_t launch_batch_start(uint64_t* t0, hipStream_t s);
hipError_t launch_batch_step(Fmt f, const BProb* probs, BState* st, const BRun& run, int grid_blocks,
                             hipStream_t s);

}  // namespace srj
