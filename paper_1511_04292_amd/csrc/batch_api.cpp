// libsrj batched solves (C ABI): srj_batch_plan / srj_batch_solve / srj_batch_destroy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/srj.h"
#include "batch.h"
#include "kernels.h"
#include "planner.h"
#include "schedule_build.h"
#include "tb_core.h"

using namespace srj;

// Set by api.cpp's error reporting helpers.
extern "C" const char* srj_last_error(void);
namespace srj {
srj_status report(srj_status s, const std::string& msg);
}

namespace {

#define BCHK(expr)                                                                             \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return report(SRJ_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int64_t kAlign = 512;

// Output rows per tile.  Tall tiles waste fewer halo rows (a tile of H output rows computes
// H + 2T rows); short tiles give a problem more waves and each wave a shorter pipeline.  The
// solve picks, whenever it rebuilds the work list, the tallest height in [kHmin, hmax] that
// still gives the running problems at least `tiles_target` tiles, so that launches stay wide
// while many problems run and become short once few remain.
constexpr int kHmin = 16;
constexpr int kHmaxDefault = 128;  // largest tile height before tuning
constexpr int kTilesTarget = 4096;  // tiles a work list aims for

int tiles_of(const Geo& g, int strip_w, int H)
{
    return (int)((g.nx + strip_w - 1) / strip_w) * (int)((g.ny + H - 1) / H);
}

struct Sched {
    std::vector<double> w;
    std::vector<int64_t> q;
    std::vector<int32_t> seq;
    int64_t M = 0;
    std::string err;
    srj_status st = SRJ_OK;
};

// Schedule of one problem, as srj_plan builds it.
void build_one(const srj_grid& g, const srj_schedule& sc, Sched* out)
{
    SchedOut o;
    out->st = make_schedule(2, g.n, nullptr, &sc, false, &o, &out->err);
    if (out->st != SRJ_OK) return;
    out->w.assign(o.omega, o.omega + o.P);
    out->q.assign(o.q, o.q + o.P);
    out->seq = std::move(o.seq);
    out->M = o.M;
}

}  // namespace

struct srj_batch_s {
    int count = 0;
    Fmt fmt = FMT_F32;
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;  // internal, capturable
    std::vector<srj_grid> grids;
    std::vector<Geo> geos;
    std::vector<BProb> probs;      // host copy (device pointers inside)
    std::vector<int32_t> M;
    int nitems = 0, npart = 0;
    void* pool = nullptr;
    BProb* probs_d = nullptr;
    BState* st_d = nullptr;
    BItem* items_d = nullptr;
    int* nitems_d = nullptr;
    double* coef_d = nullptr;
    double* partials_d = nullptr;
    double* bt2_d = nullptr;  // 2 doubles per problem
    int* remaining_d = nullptr;
    uint64_t* t0_d = nullptr;
    int* remaining_h = nullptr;  // two pinned slots: counts read back after alternate replays
    hipEvent_t ev[2] = {nullptr, nullptr};
    int* nitems_h = nullptr;  // pinned staging of the work-list length
    int items_h_len = 0;
    int hmax = 128;           // largest tile height (srj_batch_tune may change it)
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

namespace {

void destroy_batch(srj_batch_t b)
{
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    void* ptrs[] = {b->pool, b->probs_d, b->st_d, b->items_d, b->nitems_d, b->coef_d, b->partials_d,
                    b->bt2_d, b->remaining_d, b->t0_d};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (b->remaining_h) (void)hipHostFree(b->remaining_h);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
    if (b->nitems_h) (void)hipHostFree(b->nitems_h);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace

extern "C" {

srj_status srj_batch_plan(int32_t count, const srj_grid* grids, const srj_schedule* schedules, void* stream,
                          srj_batch_t* out)
{
    if (!grids || !schedules || !out || count < 1) return report(SRJ_EINVAL, "bad batch arguments");
    *out = nullptr;
    const int dt = grids[0].dtype;
    for (int j = 0; j < count; ++j) {
        const srj_grid& g = grids[j];
        if (g.ndim != 2) return report(SRJ_EINVAL, "batched problems are 2D");
        if (g.n[0] < 1 || g.n[1] < 1 || g.n[0] > (1 << 20) || g.n[1] > (1 << 20))
            return report(SRJ_EINVAL, "n must be in [1, 2^20]");
        if (!(g.h[0] > 0) || !std::isfinite(g.h[0])) return report(SRJ_EINVAL, "h must be positive");
        if (g.h[1] != g.h[0]) return report(SRJ_EINVAL, "batched problems need equal spacings (h[0] == h[1])");
        if (g.bc != 0) return report(SRJ_EINVAL, "batched problems need Dirichlet boundaries");
        if (g.dtype != dt || dt < 0 || dt > 2) return report(SRJ_EINVAL, "one storage format per batch");
    }
    srj_batch_t b = new (std::nothrow) srj_batch_s();
    if (!b) return report(SRJ_ENOMEM, "host allocation failed");
    b->count = count;
    b->fmt = (Fmt)dt;
    b->hmax = kHmaxDefault;
    b->user_stream = (hipStream_t)stream;
    b->grids.assign(grids, grids + count);
    // schedules, in parallel host threads
    std::vector<Sched> sch(count);
    {
        const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
        std::atomic<int> next{0};
        std::vector<std::thread> th;
        for (unsigned t = 0; t < nt; ++t)
            th.emplace_back([&]() {
                for (int j = next++; j < count; j = next++) build_one(grids[j], schedules[j], &sch[j]);
            });
        for (auto& t : th) t.join();
    }
    for (int j = 0; j < count; ++j)
        if (sch[j].st != SRJ_OK) {
            destroy_batch(b);
            return report(sch[j].st, "problem " + std::to_string(j) + ": " + sch[j].err);
        }
    // layout: one pool; every field of problem j shares the pitch px_j, and interior column 1
    // of every row starts on a 512-byte boundary
    const size_t es = fmt_size(b->fmt);
    std::vector<size_t> off_u0(count), off_u1(count), off_b(count), off_d0(count), off_d1(count), off_r(count);
    size_t cur = 0;
    auto carve = [&](size_t elems, size_t esize) {
        // origin = start + (kAlign/esize - 1) elements, start 512-aligned
        cur = (cur + kAlign - 1) / kAlign * kAlign;
        const size_t origin = cur + (kAlign / esize - 1) * esize;
        cur += (kAlign / esize - 1) * esize + elems * esize;
        return origin;
    };
    b->geos.resize(count);
    std::vector<double> coef;
    b->probs.resize(count);
    const int T = batch_fuse();
    const int SW = 128 - 2 * T;
    int npart = 0;
    for (int j = 0; j < count; ++j) {
        Geo& g = b->geos[j];
        g.ndim = 2;
        g.nx = grids[j].n[0];
        g.ny = grids[j].n[1];
        g.nz = 1;
        g.px = (g.nx + 2 + 63) / 64 * 64;
        g.py = g.ny + 2;
        g.wy = g.wz = 1.0;  // equal spacings
        g.dg = 4.0;
        g.bc = 0;
        const size_t elems = (size_t)(g.px * g.py);
        off_u0[j] = carve(elems, 8);
        off_u1[j] = carve(elems, 8);
        off_b[j] = carve(elems, 8);
        off_d0[j] = carve(elems, es);
        off_d1[j] = carve(elems, es);
        off_r[j] = carve(elems, es);
        BProb& P = b->probs[j];
        std::memset(&P, 0, sizeof(P));
        P.nx = (int32_t)g.nx;
        P.ny = (int32_t)g.ny;
        P.px = g.px;
        P.M = (int32_t)sch[j].M;
        P.coff = (int32_t)coef.size();
        for (int64_t k = 0; k < sch[j].M; ++k) coef.push_back(sch[j].w[sch[j].seq[k]] / 4.0);
        P.nstrip = (int32_t)((g.nx + SW - 1) / SW);
        P.H = kHmin;
        P.ntiles = tiles_of(g, SW, kHmin);
        P.pbase = npart;
        // room for the tiles at the shortest height and for the start residual's blocks
        npart += std::max<int>(P.ntiles, residual_blocks(g));
        b->nitems += P.ntiles;
        b->M.push_back(P.M);
    }
    b->npart = npart;
    cur += kAlign;  // slack after the last field: tiles may read one element past a ring
    if (hipMalloc(&b->pool, cur) != hipSuccess) {
        destroy_batch(b);
        return report(SRJ_ENOMEM, "batch pool of " + std::to_string(cur) + " bytes");
    }
    char* base = (char*)b->pool;
    for (int j = 0; j < count; ++j) {
        BProb& P = b->probs[j];
        P.u64[0] = (double*)(base + off_u0[j]);
        P.u64[1] = (double*)(base + off_u1[j]);
        P.b64 = (double*)(base + off_b[j]);
        P.d[0] = base + off_d0[j];
        P.d[1] = base + off_d1[j];
        P.rlo = base + off_r[j];
    }
    bool ok = hipMalloc(&b->probs_d, sizeof(BProb) * count) == hipSuccess &&
              hipMalloc(&b->st_d, sizeof(BState) * count) == hipSuccess &&
              hipMalloc(&b->items_d, sizeof(BItem) * (size_t)b->nitems) == hipSuccess &&
              hipMalloc(&b->nitems_d, sizeof(int)) == hipSuccess &&
              hipMalloc(&b->coef_d, sizeof(double) * std::max<size_t>(1, coef.size())) == hipSuccess &&
              hipMalloc(&b->partials_d, sizeof(double) * 2 * (size_t)npart) == hipSuccess &&
              hipMalloc(&b->bt2_d, sizeof(double) * 2 * count) == hipSuccess &&
              hipMalloc(&b->remaining_d, sizeof(int)) == hipSuccess &&
              hipMalloc(&b->t0_d, sizeof(uint64_t)) == hipSuccess &&
              hipHostMalloc(&b->remaining_h, 2 * sizeof(int), hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&b->ev[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b->ev[1], hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc(&b->nitems_h, sizeof(int), hipHostMallocDefault) == hipSuccess &&
              hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) == hipSuccess;
    if (!ok) {
        destroy_batch(b);
        return report(SRJ_ENOMEM, "batch scratch allocation failed");
    }
    for (int j = 0; j < count; ++j) b->probs[j].bt2 = b->bt2_d + 2 * j;
    if (hipMemcpy(b->coef_d, coef.data(), sizeof(double) * coef.size(), hipMemcpyHostToDevice) != hipSuccess) {
        destroy_batch(b);
        return report(SRJ_EHIP, "batch table upload failed");
    }
    *out = b;
    return SRJ_OK;
}

void srj_batch_destroy(srj_batch_t b)
{
    if (b && b->stream) (void)hipStreamSynchronize(b->stream);
    destroy_batch(b);
}

srj_status srj_batch_tune(srj_batch_t b, srj_tune_info* info)
{
    if (!b) return report(SRJ_EINVAL, "null batch");
    hipStream_t s = b->stream;
    if (b->user_stream) BCHK(hipStreamSynchronize(b->user_stream));
    const int T = batch_fuse();
    const int SW = 128 - 2 * T;
    // every problem sweeping from zero corrections, never reaching the end of an inner solve
    std::vector<BState> st(b->count);
    double pts = 0;
    for (int j = 0; j < b->count; ++j) {
        std::memset(&st[j], 0, sizeof(BState));
        st[j].phase = BP_SWEEP;
        BProb& P = b->probs[j];
        P.inner_total = 1 << 30;
        BCHK(launch_zero(b->fmt, P.d[0], b->geos[j], s));
        BCHK(launch_zero(b->fmt, P.d[1], b->geos[j], s));
        BCHK(launch_zero(b->fmt, P.rlo, b->geos[j], s));
        pts += (double)b->geos[j].nx * (double)b->geos[j].ny;
    }
    BCHK(hipMemcpyAsync(b->st_d, st.data(), sizeof(BState) * b->count, hipMemcpyHostToDevice, s));
    BRun run;
    std::memset(&run, 0, sizeof(run));
    run.tol = 0;
    run.max_outer = 0;
    run.items = b->items_d;
    run.nitems = b->nitems_d;
    run.coef = b->coef_d;
    run.partials = b->partials_d;
    run.remaining = b->remaining_d;
    const int gs = std::max(1, std::min((b->nitems + 3) / 4, 2048));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BCHK(hipEventCreate(&e0));
    BCHK(hipEventCreate(&e1));
    const int cands[] = {b->hmax, 32, 64, 128, 256};
    double before = 0, best = 0;
    int pick = b->hmax, ncand = 0;
    srj_status result = SRJ_OK;
    for (int c = 0; c < 5 && result == SRJ_OK; ++c) {
        const int H = cands[c];
        if (c > 0 && H == cands[0]) continue;
        std::vector<BItem> items;
        for (int j = 0; j < b->count; ++j) {
            BProb& P = b->probs[j];
            P.H = std::max(kHmin, std::min(H, tb_max_rows(P.px, (int)fmt_size(b->fmt))));
            P.ntiles = tiles_of(b->geos[j], SW, P.H);
            for (int t = 0; t < P.ntiles; ++t) items.push_back(BItem{j, t});
        }
        *b->nitems_h = (int)items.size();
        if (hipMemcpyAsync(b->probs_d, b->probs.data(), sizeof(BProb) * b->count, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(b->items_d, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(b->nitems_d, b->nitems_h, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            result = report(SRJ_EHIP, "batch tuning upload failed");
            break;
        }
        // 2 warm-up launches, then 6 timed (60 sweeps of every problem)
        bool ok = true;
        for (int it = 0; it < 8 && ok; ++it) {
            if (it == 2) ok = hipEventRecord(e0, s) == hipSuccess;
            ok = ok && launch_batch_step(b->fmt, b->probs_d, b->st_d, run, gs, s) == hipSuccess;
        }
        float ms = 0;
        ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (!ok) {
            result = report(SRJ_EHIP, "batch tuning launch failed");
            break;
        }
        const double us = ms * 1e3 / (6.0 * T);
        ncand += 1;
        // keep the height in place unless another one is clearly faster (3%)
        const double score = (c == 0) ? us : us * 1.03;
        if (c == 0) before = us;
        if (c == 0 || score < best) {
            best = score;
            pick = H;
        }
    }
    if (pick != cands[0]) best /= 1.03;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != SRJ_OK) return result;
    b->hmax = pick;
    if (info) {
        info->fused_sweeps = T;
        info->seg_rows = pick;
        info->candidates = ncand;
        info->us_per_sweep = best;
        info->us_per_sweep_before = before;
    }
    (void)pts;
    return SRJ_OK;
}

srj_status srj_batch_solve(srj_batch_t b, double* const* u, const double* const* f, double tol,
                           int32_t inner_cycles, int32_t max_outer, srj_solve_info* infos, double* seconds)
{
    if (!b || !u || !f) return report(SRJ_EINVAL, "null argument");
    if (!(tol >= 0) || inner_cycles < 1 || max_outer < 0) return report(SRJ_EINVAL, "bad refinement parameters");
    for (int j = 0; j < b->count; ++j)
        if (!u[j] || !f[j]) return report(SRJ_EINVAL, "null problem array");
    hipStream_t s = b->stream;
    if (b->user_stream) BCHK(hipStreamSynchronize(b->user_stream));
    BCHK(hipDeviceSynchronize());
    // inputs into the pool; ||b~||^2 per problem
    for (int j = 0; j < b->count; ++j) {
        const Geo& g = b->geos[j];
        BProb& P = b->probs[j];
        P.inner_total = inner_cycles * P.M;
        const double hh = b->grids[j].h[0] * b->grids[j].h[0];
        BCHK(launch_copy_in(FMT_F64, u[j], P.u64[0], g, s));
        BCHK(launch_copy_in(FMT_F64, u[j], P.u64[1], g, s));
        BCHK(launch_rhs(FMT_F64, f[j], hh, nullptr, P.b64, g, s));
        BCHK(launch_zero(b->fmt, P.d[0], g, s));
        BCHK(launch_zero(b->fmt, P.d[1], g, s));
        BCHK(launch_zero(b->fmt, P.rlo, g, s));
        BCHK(launch_residual(FMT_F64, P.u64[0], P.b64, g, 1, b->partials_d + 2 * P.pbase, b->bt2_d + 2 * j, s));
    }
    std::vector<double> bt2(2 * b->count);
    BCHK(hipMemcpyAsync(bt2.data(), b->bt2_d, sizeof(double) * 2 * b->count, hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    std::vector<BState> st(b->count);
    int remaining = 0;
    for (int j = 0; j < b->count; ++j) {
        std::memset(&st[j], 0, sizeof(BState));
        if (!std::isfinite(bt2[2 * j])) {
            st[j].phase = BP_DIVERGED;
            st[j].relres = NAN;
        } else if (bt2[2 * j] == 0.0) {
            // zero source and boundary: u = 0 is exact
            st[j].phase = BP_DONE;
            BCHK(launch_zero(FMT_F64, b->probs[j].u64[0], b->geos[j], s));
        } else {
            st[j].phase = BP_RESIDUAL;
            remaining += 1;
        }
    }
    BCHK(hipMemcpyAsync(b->st_d, st.data(), sizeof(BState) * b->count, hipMemcpyHostToDevice, s));
    *b->remaining_h = remaining;
    BCHK(hipMemcpyAsync(b->remaining_d, b->remaining_h, sizeof(int), hipMemcpyHostToDevice, s));
    BCHK(hipStreamSynchronize(s));

    // work list: the tiles of every running problem, at the height chosen for them
    const int T = batch_fuse();
    const int SW = 128 - 2 * T;
    const int hmax = b->hmax;
    const int tiles_target = kTilesTarget;
    std::vector<BItem> items;
    items.reserve(b->nitems);
    std::vector<int> order;
    auto running = [](const BState& x) { return x.phase == BP_SWEEP || x.phase == BP_RESIDUAL; };
    // returns true if some running problem changed its tile height
    auto build_items = [&](const std::vector<BState>& cur) {
        int H = kHmin;
        for (int h = hmax; h >= kHmin; h /= 2) {
            int64_t n = 0;
            for (int j = 0; j < b->count; ++j)
                if (running(cur[j])) n += tiles_of(b->geos[j], SW, h);
            if (n >= tiles_target) {
                H = h;
                break;
            }
        }
        bool changed = false;
        items.clear();
        order.clear();
        for (int j = 0; j < b->count; ++j) {
            if (!running(cur[j])) continue;
            BProb& P = b->probs[j];
            const int Hj = std::max(kHmin, std::min(H, tb_max_rows(P.px, (int)fmt_size(b->fmt))));
            if (P.H != Hj) {
                P.H = Hj;
                P.ntiles = tiles_of(b->geos[j], SW, Hj);
                changed = true;
            }
            order.push_back(j);
        }
        // Longest tiles first: a wave's time on a tile grows with the rows it streams (the
        // tile's output rows plus 2T), so listing the tallest tiles first lets the short ones
        // fill in behind them and ends each launch sooner (longest-processing-time-first).
        auto tile_rows = [&](int j) { return std::min<int64_t>(b->probs[j].H, b->geos[j].ny); };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            const int64_t rx = tile_rows(x), ry = tile_rows(y);
            if (rx != ry) return rx > ry;
            return b->geos[x].nx > b->geos[y].nx;
        });
        for (int j : order)
            for (int t = 0; t < b->probs[j].ntiles; ++t) items.push_back(BItem{j, t});
        b->items_h_len = (int)items.size();
        return changed;
    };
    build_items(st);
    BCHK(hipMemcpyAsync(b->probs_d, b->probs.data(), sizeof(BProb) * b->count, hipMemcpyHostToDevice, s));
    if (!items.empty())
        BCHK(hipMemcpyAsync(b->items_d, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice, s));
    *b->nitems_h = b->items_h_len;
    BCHK(hipMemcpyAsync(b->nitems_d, b->nitems_h, sizeof(int), hipMemcpyHostToDevice, s));
    BCHK(hipStreamSynchronize(s));

    BRun run;
    std::memset(&run, 0, sizeof(run));
    run.tol = tol;
    run.max_outer = max_outer;
    run.items = b->items_d;
    run.nitems = b->nitems_d;
    run.coef = b->coef_d;
    run.partials = b->partials_d;
    run.remaining = b->remaining_d;
    // One graph = G launches over a grid of gs blocks (4 waves each, grid-stride over the
    // work list).  The graph is captured again with a smaller grid whenever the work list has
    // shrunk to less than half of what the current grid covers, so that launches near the end
    // do not start thousands of waves that find no tile.
    const int G = 16;
    auto grid_for = [](int nitems) { return std::max(1, std::min((nitems + 3) / 4, 2048)); };
    int gs = 0;
    auto capture = [&](int blocks) -> srj_status {
        if (b->exec) {
            (void)hipGraphExecDestroy(b->exec);
            b->exec = nullptr;
        }
        if (b->graph) {
            (void)hipGraphDestroy(b->graph);
            b->graph = nullptr;
        }
        BCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        for (int it = 0; it < G; ++it) {
            if (launch_batch_step(b->fmt, b->probs_d, b->st_d, run, blocks, s) != hipSuccess) {
                hipGraph_t g0 = nullptr;
                (void)hipStreamEndCapture(s, &g0);
                if (g0) (void)hipGraphDestroy(g0);
                return report(SRJ_EHIP, "batch launch during capture failed");
            }
        }
        BCHK(hipStreamEndCapture(s, &b->graph));
        BCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        gs = blocks;
        return SRJ_OK;
    };
    {
        const srj_status cs = capture(grid_for(b->items_h_len));
        if (cs != SRJ_OK) return cs;
    }
    // launches needed at most: every outer step of the longest problem (its sweeps and its
    // residual) plus the first residual
    int64_t max_inner = 0;
    for (int j = 0; j < b->count; ++j) max_inner = std::max<int64_t>(max_inner, b->probs[j].inner_total);
    const int64_t cap_launches = ((int64_t)max_outer + 1) * ((max_inner + T - 1) / T + 1) + 2;
    const int64_t cap_replays = cap_launches / G + 2;
    BCHK(launch_batch_start(b->t0_d, s));
    // The host keeps one replay queued behind the one whose count of running problems it
    // reads: each replay is followed by a copy of that count into its own pinned slot and an
    // event, and the host waits on the previous replay's event only, so the device never
    // idles between replays.  At most one replay more than needed runs; its launches find
    // every problem finished and return at once.
    int64_t replays = 0;
    int listed = remaining;  // running problems when the work list was last built
    int slot = 0;
    bool pending = false;    // a replay is queued whose count has not been read yet
    while (remaining > 0 && replays < cap_replays) {
        BCHK(hipGraphLaunch(b->exec, s));
        BCHK(hipMemcpyAsync(b->remaining_h + slot, b->remaining_d, sizeof(int), hipMemcpyDeviceToHost, s));
        BCHK(hipEventRecord(b->ev[slot], s));
        replays += 1;
        if (!pending) {
            pending = true;
            slot ^= 1;
            continue;
        }
        // read the previous replay's count while this one runs
        BCHK(hipEventSynchronize(b->ev[slot ^ 1]));
        remaining = b->remaining_h[slot ^ 1];
        slot ^= 1;
        if (remaining > 0 && 4 * remaining <= 3 * listed) {
            // drop finished problems from the work list (after the queued replay)
            BCHK(hipStreamSynchronize(s));
            pending = false;
            remaining = b->remaining_h[slot ^ 1];
            if (remaining == 0) break;
            BCHK(hipMemcpyAsync(st.data(), b->st_d, sizeof(BState) * b->count, hipMemcpyDeviceToHost, s));
            BCHK(hipStreamSynchronize(s));
            if (build_items(st))
                BCHK(hipMemcpyAsync(b->probs_d, b->probs.data(), sizeof(BProb) * b->count, hipMemcpyHostToDevice, s));
            BCHK(hipMemcpyAsync(b->items_d, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice, s));
            *b->nitems_h = b->items_h_len;
            BCHK(hipMemcpyAsync(b->nitems_d, b->nitems_h, sizeof(int), hipMemcpyHostToDevice, s));
            BCHK(hipStreamSynchronize(s));
            listed = remaining;
            if (2 * grid_for(b->items_h_len) <= gs) {
                const srj_status cs = capture(grid_for(b->items_h_len));
                if (cs != SRJ_OK) return cs;
            }
        }
    }
    BCHK(hipStreamSynchronize(s));
    BCHK(hipMemcpyAsync(st.data(), b->st_d, sizeof(BState) * b->count, hipMemcpyDeviceToHost, s));
    uint64_t t0 = 0;
    BCHK(hipMemcpyAsync(&t0, b->t0_d, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    BCHK(hipStreamSynchronize(s));
    int dev = 0, rate_khz = 0;
    BCHK(hipGetDevice(&dev));
    BCHK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    srj_status worst = SRJ_OK;
    for (int j = 0; j < b->count; ++j) {
        const BProb& P = b->probs[j];
        srj_status sj;
        switch (st[j].phase) {
        case BP_DONE: sj = SRJ_OK; break;
        case BP_DIVERGED: sj = SRJ_EDIVERGED; break;
        default: sj = SRJ_ENOCONV; break;
        }
        if (sj != SRJ_EDIVERGED) BCHK(launch_copy_out(FMT_F64, P.u64[st[j].ucur], u[j], b->geos[j], s));
        if (infos) {
            infos[j].sweeps = (int64_t)st[j].outer * P.inner_total;
            infos[j].cycles = st[j].outer;
            infos[j].relres = st[j].relres;
            infos[j].seconds = (sj == SRJ_OK && st[j].t_end > t0 && rate_khz > 0)
                                   ? (double)(st[j].t_end - t0) / (rate_khz * 1e3)
                                   : 0.0;
            infos[j].status = (int32_t)sj;
        }
        if (seconds)
            seconds[j] = (sj == SRJ_OK && st[j].t_end > t0 && rate_khz > 0)
                             ? (double)(st[j].t_end - t0) / (rate_khz * 1e3)
                             : 0.0;
        if (sj == SRJ_EDIVERGED || (sj == SRJ_ENOCONV && worst == SRJ_OK)) worst = sj;
    }
    BCHK(hipStreamSynchronize(s));
    if (worst != SRJ_OK) return report(worst, "some batched problems did not converge");
    return SRJ_OK;
}

}  // extern "C"
