// libsrj C ABI: plans, solves, residuals and iterative refinement on one gfx950 GPU.
// See include/srj.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/srj.h"
#include "kernels.h"
#include "planner.h"
#include "schedule_build.h"

using namespace srj;

namespace {

thread_local std::string g_err;

srj_status fail(srj_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(SRJ_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

constexpr int64_t kAlignBytes = 512;

// A field in one storage format: origin points at element (0, 0, 0); the allocation is
// shifted so that interior column 1 of every row starts on a 512-byte boundary.
struct DField {
    void* alloc = nullptr;
    void* origin = nullptr;
};

}  // namespace

namespace srj {
// Error reporting shared with the batched entry points.
srj_status report(srj_status s, const std::string& msg) { return fail(s, msg); }

srj_status make_schedule(int d, const int64_t* n, const double* wt, const srj_schedule* sc, bool peaks,
                         SchedOut* out, std::string* err, SpecKind kind)
{
    const bool neumann = kind == SPEC_NEUMANN;
    auto bad = [&](srj_status st, const std::string& m) {
        *err = m;
        return st;
    };
    const double kmax_grid = kind == SPEC_OPERATOR ? 2.0 : neumann ? neumann_kappa_max(d, n, wt) : grid_kappa_max(d, n, wt);
    if (sc->kappa_min > 0 && sc->n_eff > 0) return bad(SRJ_EINVAL, "give kappa_min or n_eff, not both");
    if (sc->kappa_min < 0 || sc->n_eff < 0 || !std::isfinite(sc->kappa_min) || !std::isfinite(sc->n_eff))
        return bad(SRJ_EINVAL, "kappa_min and n_eff must be finite and >= 0");
    if (sc->n_eff > 0 && !(sc->n_eff > 1)) return bad(SRJ_EINVAL, "n_eff must exceed 1");
    if (sc->kappa_min > 0) {
        out->kappa_min = sc->kappa_min;
    } else if (sc->n_eff > 0) {
        // the Neumann table row for resolution N (Eq. boundaries): sin^2(pi / (2N))
        const double v = std::sin(3.14159265358979323846 / (2.0 * sc->n_eff));
        out->kappa_min = v * v;
    } else if (kind == SPEC_OPERATOR) {
        return bad(SRJ_EINVAL, "an operator's schedule needs kappa_min, n_eff or explicit weights");
    } else {
        out->kappa_min = neumann ? neumann_kappa_min(d, n, wt) : grid_kappa_min(d, n, wt);
    }
    out->kappa_max = 2.0;
    if (!(out->kappa_min < out->kappa_max)) return bad(SRJ_EINVAL, "kappa_min must be below 2");
    if (sc->P < 1 || sc->P > SRJ_MAX_LEVELS) return bad(SRJ_EINVAL, "P must be in [1, 16]");
    if (sc->q_rounding < 0 || sc->q_rounding > 3) return bad(SRJ_EINVAL, "q_rounding must be 0, 1, 2 or 3");
    const int P = sc->P;
    out->P = P;
    if (sc->omega) {
        if (!sc->q) return bad(SRJ_EINVAL, "explicit weights need counts q");
        for (int i = 0; i < P; ++i) {
            if (!std::isfinite(sc->omega[i]) || sc->omega[i] <= 0) return bad(SRJ_EINVAL, "weights must be positive");
            if (i > 0 && !(sc->omega[i] < sc->omega[i - 1]))
                return bad(SRJ_EINVAL, "weights must be strictly descending");
            if (sc->q[i] < 1) return bad(SRJ_EINVAL, "counts must be >= 1");
            out->omega[i] = sc->omega[i];
            out->q[i] = sc->q[i];
            out->beta[i] = 0.0;
        }
    } else {
        Optimum o;
        std::string e2;
        if (!optimal_schedule(P, out->kappa_min, out->kappa_max, &o, &e2))
            return bad(SRJ_ESCHEDULE, "schedule optimiser: " + e2);
        if (sc->q_rounding == 3 && P > 12) return bad(SRJ_EINVAL, "q_rounding 3 needs P <= 12");
        std::vector<int64_t> qq = round_counts(o.beta, sc->q_rounding, o.w.data(), out->kappa_min, out->kappa_max);
        if ((int)qq.size() != P) return bad(SRJ_EINVAL, "integer counts could not be formed");
        for (int i = 0; i < P; ++i) {
            out->omega[i] = o.w[i];
            out->beta[i] = o.beta[i];
            out->q[i] = qq[i];
        }
    }
    out->M = 0;
    for (int i = 0; i < P; ++i) out->M += out->q[i];
    if (sc->ordering == 2) {
        if (!sc->sequence || sc->M != out->M) return bad(SRJ_EINVAL, "explicit sequence must have M entries");
        std::vector<int64_t> cnt(P, 0);
        for (int64_t k = 0; k < out->M; ++k) {
            const int32_t i = sc->sequence[k];
            if (i < 0 || i >= P) return bad(SRJ_EINVAL, "sequence index out of range");
            cnt[i]++;
        }
        for (int i = 0; i < P; ++i)
            if (cnt[i] != out->q[i]) return bad(SRJ_EINVAL, "sequence counts differ from q");
        out->seq.assign(sc->sequence, sc->sequence + out->M);
    } else if (sc->ordering == 0 || sc->ordering == 1) {
        out->seq = order_steps(P, out->omega, out->q, out->kappa_min, out->kappa_max, sc->ordering);
    } else {
        return bad(SRJ_EINVAL, "ordering must be 0, 1 or 2");
    }
    // convergence of the integer scheme on the grid's own spectrum (Sec. 4.3)
    out->gamma_q = gamma_q_max(P, out->omega, out->q, out->kappa_min,
                               std::max(kmax_grid, out->kappa_min * 1.0000001));
    if (!(out->gamma_q < 1.0))
        return bad(SRJ_ESCHEDULE, "integer scheme not convergent: max Gamma_q = " + std::to_string(out->gamma_q));
    if (peaks) partial_peaks(P, out->omega, out->seq, out->kappa_min, out->kappa_max, &out->pre, &out->suf);
    double r = 0;
    for (int i = 0; i < P; ++i) r += out->omega[i] * (double)out->q[i];
    out->rho = r / (double)out->M;
    return SRJ_OK;
}
}  // namespace srj

struct srj_plan_s {
    srj_grid grid{};
    bool iso = true;  // equal spacings: the temporally blocked kernels apply
    double hh = 0;    // h_x^2, the scale of b
    Fmt fmt = FMT_F64;
    hipStream_t stream = nullptr;
    Geo geo{};
    size_t field_elems = 0;  // elements per allocation (including alignment slack)

    // schedule
    int P = 0;
    double omega[SRJ_MAX_LEVELS] = {0};
    double beta[SRJ_MAX_LEVELS] = {0};
    int64_t q[SRJ_MAX_LEVELS] = {0};
    int64_t M = 0;
    std::vector<int32_t> seq;
    std::vector<double> cseq;  // c_k = w_seq[k] / (2d)
    double kappa_min = 0, kappa_max = 0, rho = 0, gamma_q = 0, pre = 0, suf = 0;
    int fuse = 8;
    int seg_rows = 0;  // output rows per wave in the fused 2D kernel (0: from the occupancy)
    bool resident = false;      // srj_solve runs in one workgroup with the grid in LDS
    bool ldsfuse = false;       // fused sweeps run in the LDS-tiled kernel (2D binary64 plans
                                // with unequal spacings, Neumann boundaries or an operator)
    double* cseq_d = nullptr;   // the cycle's coefficients on the device (resident solves)
    uint32_t fused_launches = 0;  // fused launches so far: their parity alternates the stream direction
    bool store_nt = false;        // fused 2D binary64 stores carry the non-temporal hint

    // device buffers
    DField A, B, blo;  // iterate pair, b (or the refinement's inner right-hand side) in the sweep format
    DField b64f, x64;  // binary64 b, and the binary64 iterate of refinement / residual evaluation
    double* b64 = nullptr;  // b64f.origin
    // variable-coefficient operator plans: scaled weights, a_P and the mask (padded fields)
    DField opw[6], opap;
    void* opmask_alloc = nullptr;
    uint8_t* opmask = nullptr;
    double* partials = nullptr;
    double* dres = nullptr;   // device {sum, max}
    double* hres = nullptr;   // pinned host copy
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

srj_status alloc_field(srj_plan_t p, Fmt f, DField* d)
{
    size_t es = fmt_size(f);
    size_t bytes = p->field_elems * es;
    const hipError_t e = hipMalloc(&d->alloc, bytes);
    if (e != hipSuccess) {
        d->alloc = nullptr;
        return fail(SRJ_ENOMEM,
                    "device allocation of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    int64_t off = kAlignBytes / (int64_t)es - 1;
    d->origin = (char*)d->alloc + off * es;
    return SRJ_OK;
}

void free_field(DField* d)
{
    if (d->alloc) (void)hipFree(d->alloc);
    d->alloc = d->origin = nullptr;
}

bool is_finite(double x) { return std::isfinite(x); }

srj_status build_schedule(srj_plan_t p, const srj_schedule* sc)
{
    SchedOut o;
    std::string err;
    const double wt[3] = {p->geo.wy, p->geo.wz, p->geo.dg};
    const SpecKind kind = p->geo.op ? SPEC_OPERATOR : (p->geo.bc == 1 ? SPEC_NEUMANN : SPEC_DIRICHLET);
    srj_status st = make_schedule(p->grid.ndim, p->grid.n, p->iso ? nullptr : wt, sc, true, &o, &err, kind);
    if (st != SRJ_OK) return fail(st, err);
    p->P = o.P;
    std::memcpy(p->omega, o.omega, sizeof(o.omega));
    std::memcpy(p->beta, o.beta, sizeof(o.beta));
    std::memcpy(p->q, o.q, sizeof(o.q));
    p->M = o.M;
    p->seq = std::move(o.seq);
    p->kappa_min = o.kappa_min;
    p->kappa_max = o.kappa_max;
    p->rho = o.rho;
    p->gamma_q = o.gamma_q;
    p->pre = o.pre;
    p->suf = o.suf;
    p->cseq.resize(p->M);
    for (int64_t k = 0; k < p->M; ++k) p->cseq[k] = p->omega[p->seq[k]] / p->geo.dg;
    return SRJ_OK;
}

void destroy(srj_plan_t p)
{
    if (!p) return;
    free_field(&p->A);
    free_field(&p->B);
    free_field(&p->blo);
    free_field(&p->b64f);
    free_field(&p->x64);
    for (auto& f : p->opw) free_field(&f);
    free_field(&p->opap);
    if (p->opmask_alloc) (void)hipFree(p->opmask_alloc);
    if (p->cseq_d) (void)hipFree(p->cseq_d);
    if (p->partials) (void)hipFree(p->partials);
    if (p->dres) (void)hipFree(p->dres);
    if (p->hres) (void)hipHostFree(p->hres);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    delete p;
}

srj_status residual_now(srj_plan_t p, const void* u, Fmt f, int zero_int, double* sum, double* mx)
{
    HIPCHK(launch_residual(f, u, p->b64, p->geo, zero_int, p->partials, p->dres, p->stream));
    HIPCHK(hipMemcpyAsync(p->hres, p->dres, 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    *sum = p->hres[0];
    *mx = p->hres[1];
    return SRJ_OK;
}

// Run sweeps k0 .. k0+n-1 on the ping-pong pair; *cur is updated to the buffer holding the
// result.  Fused launches never straddle a cycle boundary.
srj_status run_sweeps(srj_plan_t p, DField** cur, DField** nxt, const void* b, int64_t k0, int64_t n,
                      int64_t* launches = nullptr)
{
    int64_t k = k0;
    const int64_t end = k0 + n;
    while (k < end) {
        if (p->fuse <= 0) {
            HIPCHK(launch_sweep_unfused(p->fmt, (*cur)->origin, (*nxt)->origin, b, p->geo,
                                        p->cseq[k % p->M], p->stream));
            k += 1;
        } else {
            int64_t to_cycle_end = p->M - (k % p->M);
            int T = (int)std::min<int64_t>({(int64_t)p->fuse, end - k, to_cycle_end});
            Coefs co;
            for (int l = 0; l < T; ++l) co.c[l] = p->cseq[(k + l) % p->M];
            if (p->ldsfuse)
                HIPCHK(launch_sweep_lds2d((*cur)->origin, (*nxt)->origin, b, p->geo, co, T, p->stream));
            else if (p->geo.ndim == 2)
                HIPCHK(launch_sweep_fused(p->fmt, (*cur)->origin, (*nxt)->origin, b, p->geo, co, T, p->seg_rows,
                                          (int)(p->fused_launches++ & 1u), p->store_nt, p->stream));
            else
                HIPCHK(launch_sweep_fused3d(p->fmt, (*cur)->origin, (*nxt)->origin, b, p->geo, co, T,
                                            (int)(p->fused_launches++ & 1u), p->stream));
            k += T;
        }
        if (launches) *launches += 1;
        std::swap(*cur, *nxt);
    }
    return SRJ_OK;
}

// b from the user's f: h_x^2 f (Poisson plans) or f / a_P (operator plans), in the sweep
// format (blo) and in binary64 (b64)
hipError_t load_rhs(srj_plan_t p, const double* f)
{
    if (p->geo.op) {
        hipError_t e = launch_op_rhs(f, (const double*)p->opap.origin, p->b64, p->geo, p->stream);
        if (e != hipSuccess) return e;
        return hipMemcpyAsync(p->blo.origin, p->b64, sizeof(double) * p->field_elems - sizeof(double) * (kAlignBytes / 8 - 1),
                              hipMemcpyDeviceToDevice, p->stream);
    }
    return launch_rhs(p->fmt, f, p->hh, p->blo.origin, p->b64, p->geo, p->stream);
}

void fill_info(srj_solve_info* info, int64_t sweeps, int64_t cycles, double relres, double sec, srj_status st)
{
    if (!info) return;
    info->sweeps = sweeps;
    info->cycles = cycles;
    info->relres = relres;
    info->seconds = sec;
    info->status = (int32_t)st;
}

// Where a solve records the relres of its checks (host memory, first cap entries kept).
struct History {
    double* out = nullptr;
    int64_t cap = 0;
    int64_t len = 0;
    void push(double rr)
    {
        if (len < cap) out[len] = rr;
        len += 1;
    }
};

// Solve on the plan's fields: A and B hold the initial state (ring included), blo/b64 the
// scaled source.  On return *cur points at the field with the returned state.
// k0 (0 <= k0 < M): the state in A/B is the iterate after k0 sweeps of a cycle; the solve
// completes that cycle before its first check.  hist (may be null) receives every check.
srj_status solve_fields(srj_plan_t p, double tol, int64_t max_sweeps, DField** cur, int64_t* k_out,
                        int64_t* cycles_out, double* rr_out, srj_status* result, int64_t k0 = 0,
                        History* hist = nullptr)
{
    if (p->resident && k0 == 0 && !hist) {
        // the whole solve in one launch, the grid in LDS; one synchronisation
        HIPCHK(launch_small_solve((const double*)p->A.origin, (const double*)p->blo.origin, (double*)p->B.origin,
                                  p->geo, p->cseq_d, p->M, tol, max_sweeps, p->dres, p->stream));
        HIPCHK(hipMemcpyAsync(p->hres, p->dres, 4 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
        HIPCHK(hipStreamSynchronize(p->stream));
        *cur = &p->B;
        *k_out = (int64_t)p->hres[0];
        *cycles_out = (int64_t)p->hres[1];
        *rr_out = p->hres[2];
        const int stt = (int)p->hres[3];
        *result = stt == 5 ? SRJ_ENOCONV : (stt == 6 ? SRJ_EDIVERGED : SRJ_OK);
        return SRJ_OK;
    }
    // reference norm: ||b~|| (the residual of the zero interior); with Neumann boundaries the
    // operator is singular and the reference is the initial residual
    double bt2, bmax;
    srj_status st = residual_now(p, p->A.origin, p->fmt, p->geo.bc == 1 ? 0 : 1, &bt2, &bmax);
    if (st != SRJ_OK) return st;
    *cur = &p->A;
    DField* nxt = &p->B;
    int64_t k = 0, cycles = 0;
    double rr = 0.0;
    *result = SRJ_OK;
    if (!is_finite(bt2)) {
        *result = SRJ_EDIVERGED;
        rr = NAN;
        if (hist) hist->push(rr);
    } else if (bt2 == 0.0) {
        // Dirichlet: zero source and zero boundary, u = 0 is exact; Neumann: the initial
        // state already has a zero residual and is returned as it is
        if (p->geo.bc == 0) HIPCHK(launch_zero(p->fmt, (*cur)->origin, p->geo, p->stream));
        rr = 0.0;
    } else {
        // Binary64 plans whose sweeps run one per launch (and single-sweep cycles) take each
        // check from the cycle's first sweep: that sweep forms the residual of the state it
        // starts from, bit for bit as a separate evaluation would, and writes its result to
        // the other field, so a converged state is still in *cur.  Blocked launches carry a
        // whole cycle's sweeps per pass over the grid, where a separate check costs less
        // than an extra unblocked sweep.
        const bool fused_check = p->fmt == FMT_F64 && (p->fuse <= 0 || p->M == 1);
        if (k0 > 0) {
            // a resumed solve: the rest of the cycle first (a mid-cycle state is not checked)
            if (p->M - k0 > max_sweeps) {
                double r2, rmax;
                if ((st = residual_now(p, (*cur)->origin, p->fmt, 0, &r2, &rmax)) != SRJ_OK) return st;
                *k_out = 0;
                *cycles_out = 0;
                *rr_out = std::sqrt(r2) / std::sqrt(bt2);
                *result = SRJ_ENOCONV;
                return SRJ_OK;
            }
            if ((st = run_sweeps(p, cur, &nxt, p->blo.origin, k0, p->M - k0)) != SRJ_OK) return st;
            k = p->M - k0;
            cycles = 1;
        }
        for (;;) {
            double r2, rmax;
            const bool room = k + p->M <= max_sweeps;  // k counts this call's sweeps
            if (fused_check && room) {
                HIPCHK(launch_sweep_residual((const double*)(*cur)->origin, (double*)nxt->origin, p->b64, p->geo,
                                             p->cseq[0], p->partials, p->dres, p->stream));
                HIPCHK(hipMemcpyAsync(p->hres, p->dres, 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
                HIPCHK(hipStreamSynchronize(p->stream));
                r2 = p->hres[0];
                rmax = p->hres[1];
            } else if ((st = residual_now(p, (*cur)->origin, p->fmt, 0, &r2, &rmax)) != SRJ_OK) {
                return st;
            }
            rr = std::sqrt(r2) / std::sqrt(bt2);
            if (hist) hist->push(rr);
            if (!is_finite(rr)) {
                *result = SRJ_EDIVERGED;
                break;
            }
            if (rr <= tol) break;
            if (!room) {
                *result = SRJ_ENOCONV;
                break;
            }
            if (fused_check) {
                std::swap(*cur, nxt);  // the cycle's first sweep is done
                if ((st = run_sweeps(p, cur, &nxt, p->blo.origin, 1, p->M - 1)) != SRJ_OK) return st;
            } else if ((st = run_sweeps(p, cur, &nxt, p->blo.origin, 0, p->M)) != SRJ_OK) {
                return st;
            }
            k += p->M;
            cycles += 1;
        }
    }
    *k_out = k;
    *cycles_out = cycles;
    *rr_out = rr;
    return SRJ_OK;
}

srj_status finish_info(srj_plan_t p, srj_solve_info* info, int64_t k, int64_t cycles, double rr, srj_status result)
{
    HIPCHK(hipEventRecord(p->ev1, p->stream));
    HIPCHK(hipEventSynchronize(p->ev1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, p->ev0, p->ev1));
    fill_info(info, k, cycles, rr, ms * 1e-3, result);
    if (result == SRJ_ENOCONV) return fail(result, "tolerance not reached within the sweep budget");
    if (result == SRJ_EDIVERGED) return fail(result, "non-finite residual");
    return SRJ_OK;
}

}  // namespace

extern "C" {

const char* srj_status_string(srj_status s)
{
    switch (s) {
    case SRJ_OK: return "ok";
    case SRJ_EINVAL: return "invalid argument";
    case SRJ_ENOMEM: return "out of memory";
    case SRJ_EHIP: return "HIP runtime error";
    case SRJ_ESCHEDULE: return "schedule error";
    case SRJ_ENOCONV: return "tolerance not reached";
    case SRJ_EDIVERGED: return "diverged";
    }
    return "unknown status";
}

const char* srj_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace {

// A plan for the Poisson operator (coef == null) or for a variable-coefficient operator
// given by the user's coefficient arrays and mask (srj_plan_operator).
srj_status create_plan(const srj_grid* grid, const srj_schedule* schedule, void* stream, const double* coef,
                       const uint8_t* mask, srj_plan_t* out)
{
    if (!grid || !schedule || !out) return fail(SRJ_EINVAL, "null argument");
    *out = nullptr;
    if (grid->ndim != 2 && grid->ndim != 3) return fail(SRJ_EINVAL, "ndim must be 2 or 3");
    for (int i = 0; i < grid->ndim; ++i) {
        if (grid->n[i] < 1 || grid->n[i] > (1 << 20)) return fail(SRJ_EINVAL, "n must be in [1, 2^20]");
        if (!(grid->h[i] > 0) || !is_finite(grid->h[i])) return fail(SRJ_EINVAL, "every h[i] must be positive");
    }
    if (grid->dtype < 0 || grid->dtype > 2) return fail(SRJ_EINVAL, "dtype must be 0, 1 or 2");
    if (grid->bc != 0 && grid->bc != 1) return fail(SRJ_EINVAL, "bc must be 0 (Dirichlet) or 1 (Neumann)");
    if (grid->bc == 1 && grid->dtype != 0) return fail(SRJ_EINVAL, "Neumann grids are binary64 only");
    if (grid->bc == 1)
        for (int i = 0; i < grid->ndim; ++i)
            if (grid->n[i] < 2) return fail(SRJ_EINVAL, "a Neumann grid needs at least 2 cells per axis");
    if (coef) {
        if (grid->dtype != 0 || grid->bc != 0)
            return fail(SRJ_EINVAL, "operator plans are binary64 with fixed (Dirichlet) boundary values");
        if (!schedule->omega && !(schedule->kappa_min > 0) && !(schedule->n_eff > 0))
            return fail(SRJ_EINVAL, "operator plans need explicit weights, kappa_min or n_eff");
    }
    srj_plan_t p = new (std::nothrow) srj_plan_s();
    if (!p) return fail(SRJ_ENOMEM, "host allocation failed");
    p->grid = *grid;
    if (grid->ndim == 2) {
        p->grid.n[2] = 1;
        p->grid.h[2] = grid->h[0];
    }
    p->fmt = (Fmt)grid->dtype;
    p->stream = (hipStream_t)stream;
    Geo& g = p->geo;
    g.ndim = grid->ndim;
    g.nx = grid->n[0];
    g.ny = grid->n[1];
    g.nz = grid->ndim == 3 ? grid->n[2] : 1;
    geo_set_weights(g, p->grid.h, &p->iso);
    g.bc = grid->bc;
    p->hh = p->grid.h[0] * p->grid.h[0];
    if (coef) {
        // the operator carries its own scaling: unit weights, b = f / a_P, c_k = w_k
        g.op = 1;
        g.wy = g.wz = 1.0;
        g.dg = 1.0;
        p->iso = false;
        p->hh = 1.0;
    }
    srj_status st = build_schedule(p, schedule);
    if (st != SRJ_OK) {
        destroy(p);
        return st;
    }
    // pitch: multiple of 512 bytes for the narrowest format used (bf16 -> 256 elements)
    const int64_t ae = kAlignBytes / 2;
    g.px = ((g.nx + 2 + ae - 1) / ae) * ae;
    g.py = g.ny + 2;
    const int64_t rows = (g.ndim == 3 ? g.nz + 2 : 1) * g.py;
    p->field_elems = (size_t)(rows * g.px + kAlignBytes);
    if ((st = alloc_field(p, p->fmt, &p->A)) != SRJ_OK || (st = alloc_field(p, p->fmt, &p->B)) != SRJ_OK ||
        (st = alloc_field(p, p->fmt, &p->blo)) != SRJ_OK) {
        destroy(p);
        return st;
    }
    // binary64 b and iterate, separate from the sweep fields in every format: refinement
    // writes its inner right-hand side into blo while b64 keeps b
    if ((st = alloc_field(p, FMT_F64, &p->b64f)) != SRJ_OK || (st = alloc_field(p, FMT_F64, &p->x64)) != SRJ_OK) {
        destroy(p);
        return st;
    }
    p->b64 = (double*)p->b64f.origin;
    if (coef) {
        const int nnb = 2 * g.ndim;
        double* wp[6] = {nullptr};
        for (int m = 0; m < nnb; ++m) {
            if ((st = alloc_field(p, FMT_F64, &p->opw[m])) != SRJ_OK) {
                destroy(p);
                return st;
            }
            wp[m] = (double*)p->opw[m].origin;
            g.w[m] = wp[m];
        }
        if ((st = alloc_field(p, FMT_F64, &p->opap)) != SRJ_OK) {
            destroy(p);
            return st;
        }
        if (mask) {
            if (hipMalloc(&p->opmask_alloc, p->field_elems) != hipSuccess) {
                destroy(p);
                return fail(SRJ_ENOMEM, "allocation of the mask field failed");
            }
            p->opmask = (uint8_t*)p->opmask_alloc + (kAlignBytes - 1);
        }
        g.mask = p->opmask;
        if (launch_op_setup(coef, mask, wp, (double*)p->opap.origin, p->opmask, g, p->stream) != hipSuccess) {
            destroy(p);
            return fail(SRJ_EHIP, "operator setup failed");
        }
    }
    const int nb = residual_blocks(g);
    if (hipMalloc(&p->partials, sizeof(double) * 2 * (size_t)nb) != hipSuccess ||
        hipMalloc(&p->dres, sizeof(double) * 4) != hipSuccess ||
        hipHostMalloc(&p->hres, sizeof(double) * 4, hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&p->ev0) != hipSuccess || hipEventCreate(&p->ev1) != hipSuccess) {
        destroy(p);
        return fail(SRJ_ENOMEM, "allocation of reduction scratch failed");
    }
    if (launch_zero(p->fmt, p->blo.origin, g, p->stream) != hipSuccess ||
        launch_zero(FMT_F64, p->b64, g, p->stream) != hipSuccess ||
        launch_zero(FMT_F64, p->x64.origin, g, p->stream) != hipSuccess) {
        destroy(p);
        return fail(SRJ_EHIP, "initial fill failed");
    }
    // 2D: 10 sweeps per launch; 3D: 5, 4 or 3 from a cost model of the launch shape (5 at 512^3,
    // where it measured 7-10% faster per sweep than 4; 4 where 5 would leave compute units
    // idle or waste much of a short z run); unequal spacings and Neumann boundaries: the
    // register-streamed kernels implement the equal-spacing Dirichlet operator only
    p->fuse = (!p->iso || g.bc != 0) ? 0
              : (g.ndim == 2)        ? kMaxFuse
                                     : (fused3d_fits(g, p->fmt) ? fused3d_default_depth(g, p->fmt) : 0);
    // 2D binary64 with unequal spacings, Neumann boundaries or an operator: up to 8 sweeps per
    // launch on tiles held in LDS (the register-streamed kernels implement the equal-spacing
    // Dirichlet operator only); in 3D these plans sweep once per launch
    p->ldsfuse = (!p->iso || g.bc != 0 || g.op) && lds_fuse_fits(g, p->fmt);
    if (p->ldsfuse) p->fuse = lds_fuse_max();
    // Fused 2D binary64 launches store with the non-temporal hint when the three fields they
    // touch (input, output, b) exceed the 256 MiB memory-side cache but fit in twice it: at
    // 4096^2 faster at every depth (2% at 10 sweeps per launch, 5% at one); at 2048^2, inside
    // the cache, as fast at 10 and 37% slower at one; from 8192^2 on slower (2-3% at 10).  The
    // 3D kernel always takes the hint, the other formats never.
    {
        const double ws = 3.0 * (double)p->field_elems * sizeof(double), mall = 256.0 * 1024.0 * 1024.0;
        p->store_nt = p->fmt == FMT_F64 && g.ndim == 2 && p->iso && g.bc == 0 && !g.op && ws > mall &&
                      ws <= 2.0 * mall;
    }
    // small binary64 2D grids: srj_solve keeps the grid in one compute unit's LDS
    if (p->fmt == FMT_F64 && small_solve_fits(g)) {
        if (hipMalloc(&p->cseq_d, sizeof(double) * (size_t)p->M) != hipSuccess ||
            hipMemcpy(p->cseq_d, p->cseq.data(), sizeof(double) * (size_t)p->M, hipMemcpyHostToDevice) != hipSuccess) {
            destroy(p);
            return fail(SRJ_ENOMEM, "allocation of the coefficient table failed");
        }
        p->resident = true;
    }
    *out = p;
    return SRJ_OK;
}

}  // namespace

extern "C" {

srj_status srj_plan(const srj_grid* grid, const srj_schedule* schedule, void* stream, srj_plan_t* out)
{
    return create_plan(grid, schedule, stream, nullptr, nullptr, out);
}

srj_status srj_plan_operator(const srj_grid* grid, const srj_schedule* schedule, const double* coef,
                             const uint8_t* mask, void* stream, srj_plan_t* out)
{
    if (!coef) return fail(SRJ_EINVAL, "null coefficients");
    return create_plan(grid, schedule, stream, coef, mask, out);
}

void srj_plan_destroy(srj_plan_t plan)
{
    if (plan) (void)hipStreamSynchronize(plan->stream);
    destroy(plan);
}

srj_status srj_plan_describe(srj_plan_t p, srj_plan_desc* out)
{
    if (!p || !out) return fail(SRJ_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->P = p->P;
    out->M = p->M;
    for (int i = 0; i < p->P; ++i) {
        out->omega[i] = p->omega[i];
        out->beta[i] = p->beta[i];
        out->q[i] = p->q[i];
    }
    out->kappa_min = p->kappa_min;
    out->kappa_max = p->kappa_max;
    out->rho = p->rho;
    out->gamma_q_max = p->gamma_q;
    out->prefix_peak_log10 = p->pre;
    out->suffix_peak_log10 = p->suf;
    out->fused_sweeps = p->fuse;
    out->resident = p->resident ? 1 : 0;
    out->store_nt = p->store_nt ? 1 : 0;
    return SRJ_OK;
}

srj_status srj_plan_sequence(srj_plan_t p, int32_t* seq, int64_t cap)
{
    if (!p || !seq) return fail(SRJ_EINVAL, "null argument");
    if (cap < p->M) return fail(SRJ_EINVAL, "capacity below M");
    std::memcpy(seq, p->seq.data(), sizeof(int32_t) * (size_t)p->M);
    return SRJ_OK;
}

srj_status srj_plan_set_fusion(srj_plan_t p, int32_t fused, int32_t seg_rows)
{
    if (!p) return fail(SRJ_EINVAL, "null plan");
    if (fused < 0 || fused > kMaxFuse) return fail(SRJ_EINVAL, "fusion depth must be in [0, 10]");
    if (p->geo.ndim == 3 && fused > kMaxFuse3d) return fail(SRJ_EINVAL, "3D fusion depth must be in [0, 5]");
    if (fused > 0 && (!p->iso || p->geo.bc != 0 || p->geo.op)) {
        if (!p->ldsfuse)
            return fail(SRJ_EINVAL, "fused sweeps with unequal spacings, Neumann boundaries or an operator need a 2D "
                                    "binary64 plan");
        if (fused > lds_fuse_max())
            return fail(SRJ_EINVAL, "at most 8 fused sweeps with unequal spacings, Neumann boundaries or an operator");
    }
    if (p->geo.ndim == 3 && fused > 0 && !fused3d_fits(p->geo, p->fmt))
        return fail(SRJ_EINVAL, "z planes too large for the fused 3D kernel (1 GiB per plane at most)");
    if (seg_rows < 0 || seg_rows > (1 << 20)) return fail(SRJ_EINVAL, "segment rows must be in [0, 2^20]");
    p->fuse = fused;
    p->seg_rows = seg_rows;
    p->resident = false;  // an explicit launch shape: srj_solve runs the sweep kernels
    return SRJ_OK;
}

srj_status srj_residual(srj_plan_t p, const double* u, const double* f, double* r_out, double norms[4])
{
    if (!p || !u || !f || !norms) return fail(SRJ_EINVAL, "null argument");
    srj_status st;
    // u goes to the plan's binary64 iterate field; b to b64 (and blo, as a solve would)
    HIPCHK(launch_copy_in(FMT_F64, u, p->x64.origin, p->geo, p->stream));
    HIPCHK(load_rhs(p, f));
    double s0, m0, s1, m1;
    if ((st = residual_now(p, p->x64.origin, FMT_F64, 1, &s0, &m0)) != SRJ_OK) return st;
    if (r_out) HIPCHK(launch_residual_out((const double*)p->x64.origin, p->b64, r_out, p->geo, p->stream));
    if ((st = residual_now(p, p->x64.origin, FMT_F64, 0, &s1, &m1)) != SRJ_OK) return st;
    norms[0] = std::sqrt(s1);
    norms[1] = m1;
    norms[2] = std::sqrt(s0);
    norms[3] = s0 > 0 ? std::sqrt(s1) / std::sqrt(s0) : 0.0;
    return SRJ_OK;
}

srj_status srj_sweeps(srj_plan_t p, double* u, const double* f, int64_t k0, int64_t n, double* stats)
{
    if (!p || !u || !f) return fail(SRJ_EINVAL, "null argument");
    if (k0 < 0 || n < 0) return fail(SRJ_EINVAL, "k0 and nsweeps must be >= 0");
    HIPCHK(launch_copy_in(p->fmt, u, p->A.origin, p->geo, p->stream));
    HIPCHK(launch_copy_in(p->fmt, u, p->B.origin, p->geo, p->stream));
    HIPCHK(load_rhs(p, f));
    DField *cur = &p->A, *nxt = &p->B;
    int64_t launches = 0;
    HIPCHK(hipEventRecord(p->ev0, p->stream));
    srj_status st = run_sweeps(p, &cur, &nxt, p->blo.origin, k0 % p->M, n, &launches);
    if (st != SRJ_OK) return st;
    HIPCHK(hipEventRecord(p->ev1, p->stream));
    HIPCHK(launch_copy_out(p->fmt, cur->origin, u, p->geo, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    if (stats) {
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, p->ev0, p->ev1));
        stats[0] = ms * 1e-3;
        stats[1] = (double)launches;
    }
    return SRJ_OK;
}

}  // extern "C"

namespace {

struct Cand {
    int T, H;
};

// Launch shapes the tuner times for a plan, the one in place first.
std::vector<Cand> tune_candidates(srj_plan_t p)
{
    std::vector<Cand> cands;
    cands.push_back({p->fuse, p->seg_rows});
    if (!p->iso || p->geo.bc != 0 || p->geo.op) {
        // unequal spacings, Neumann boundaries, operators: the unfused kernel, and in 2D
        // binary64 the LDS-tiled one
        if (p->ldsfuse)
            for (int T : {8, 4, 2, 0}) cands.push_back({T, 0});
    } else if (p->geo.ndim == 2) {
        for (int T : {10, 8, 6, 4})
            for (int H : {0, 24, 32, 48, 64, 96, 128}) cands.push_back({T, H});
    } else {
        if (fused3d_fits(p->geo, p->fmt))
            for (int T : {5, 4, 3, 2, 1}) cands.push_back({T, 0});
        cands.push_back({0, 0});
    }
    return cands;
}

// Cache key of a plan's tuning: device, grid, format, boundary kind, spacing kind, operator,
// and the cycle length M (launches end at cycle ends, so M shapes the launches timed).
srj_status tune_key(srj_plan_t p, std::string* key)
{
    int dev = 0;
    hipDeviceProp_t prop;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    std::string arch(prop.gcnArchName);
    for (char& c : arch)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    if (arch.empty()) arch = "unknown";
    *key = arch + " " + std::to_string(prop.multiProcessorCount) + " " + std::to_string(p->geo.ndim) + " " +
           std::to_string(p->geo.nx) + " " + std::to_string(p->geo.ny) + " " + std::to_string(p->geo.nz) + " " +
           std::to_string((int)p->fmt) + " " + std::to_string(p->geo.bc) + " " + std::to_string(p->iso ? 1 : 0) +
           " " + std::to_string(p->geo.op ? 1 : 0) + " " + std::to_string(p->M);
    return SRJ_OK;
}

constexpr const char* kTuneTag = "srj-tune-v2";

}  // namespace

extern "C" {

srj_status srj_plan_tune(srj_plan_t p, srj_tune_info* info)
{
    if (!p) return fail(SRJ_EINVAL, "null plan");
    std::vector<Cand> cands = tune_candidates(p);
    HIPCHK(launch_zero(p->fmt, p->A.origin, p->geo, p->stream));
    HIPCHK(launch_zero(p->fmt, p->B.origin, p->geo, p->stream));
    // device time per sweep of a configuration: a unit of sweeps that is a whole number of
    // launches at every candidate depth (lcm of {10, 8, 6, 4} in 2D, of {5, 4, 3, 2, 1} in
    // 3D), repeated until the timed run lasts about a millisecond
    const int64_t unit = (p->geo.ndim == 2) ? 120 : 60;
    auto time_one = [&](const Cand& c, double* us) -> srj_status {
        p->fuse = c.T;
        p->seg_rows = c.H;
        DField *cur = &p->A, *nxt = &p->B;
        srj_status st = run_sweeps(p, &cur, &nxt, p->blo.origin, 0, unit);  // warm-up
        if (st != SRJ_OK) return st;
        int64_t n = unit;
        for (int rep = 0; rep < 4; ++rep) {
            HIPCHK(hipEventRecord(p->ev0, p->stream));
            st = run_sweeps(p, &cur, &nxt, p->blo.origin, 0, n);
            if (st != SRJ_OK) return st;
            HIPCHK(hipEventRecord(p->ev1, p->stream));
            HIPCHK(hipEventSynchronize(p->ev1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, p->ev0, p->ev1));
            *us = ms * 1e3 / (double)n;
            if (ms >= 1.0f || n >= unit * 64) break;
            n = std::min<int64_t>(unit * 64, n * (int64_t)std::ceil(1.2 / std::max(ms, 0.01f)));
            n = (n + unit - 1) / unit * unit;
        }
        return SRJ_OK;
    };
    double before = 0, best = 0;
    Cand pick = cands[0];
    for (size_t i = 0; i < cands.size(); ++i) {
        double us = 0;
        srj_status st = time_one(cands[i], &us);
        if (st != SRJ_OK) {
            p->fuse = cands[0].T;
            p->seg_rows = cands[0].H;
            return st;
        }
        if (i == 0) before = us;
        // the configuration in place stays unless another one is clearly faster (3%), so
        // timing noise does not flip between near-equal shapes
        const double score = (i == 0) ? us : us * 1.03;
        if (i == 0 || score < best) {
            best = score;
            pick = cands[i];
        }
    }
    best = (pick.T == cands[0].T && pick.H == cands[0].H) ? before : best / 1.03;
    p->fuse = pick.T;
    p->seg_rows = pick.H;
    if (info) {
        info->fused_sweeps = pick.T;
        info->seg_rows = pick.H;
        info->candidates = (int32_t)cands.size();
        info->us_per_sweep = best;
        info->us_per_sweep_before = before;
    }
    return SRJ_OK;
}

srj_status srj_plan_tune_cached(srj_plan_t p, const char* path, srj_tune_info* info)
{
    if (!p || !path) return fail(SRJ_EINVAL, "null argument");
    std::string key;
    srj_status st = tune_key(p, &key);
    if (st != SRJ_OK) return st;
    const std::vector<Cand> allowed = tune_candidates(p);
    // the last line for this key wins
    bool hit = false;
    Cand got{0, 0};
    double got_us = 0;
    if (FILE* fp = std::fopen(path, "r")) {
        char line[1024];
        const std::string head = std::string(kTuneTag) + " " + key + " ";
        while (std::fgets(line, sizeof line, fp)) {
            const std::string l(line);
            if (l.compare(0, head.size(), head) != 0) continue;
            int T = 0, H = 0;
            double us = 0;
            if (std::sscanf(l.c_str() + head.size(), "%d %d %lf", &T, &H, &us) != 3) continue;
            bool ok = false;
            for (const Cand& c : allowed) ok = ok || (c.T == T && c.H == H);
            if (!ok) continue;
            hit = true;
            got = {T, H};
            got_us = us;
        }
        std::fclose(fp);
    }
    if (hit) {
        p->fuse = got.T;
        p->seg_rows = got.H;
        if (info) {
            info->fused_sweeps = got.T;
            info->seg_rows = got.H;
            info->candidates = 0;
            info->us_per_sweep = got_us;
            info->us_per_sweep_before = got_us;
        }
        return SRJ_OK;
    }
    srj_tune_info ti;
    if ((st = srj_plan_tune(p, &ti)) != SRJ_OK) return st;
    if (info) *info = ti;
    FILE* fp = std::fopen(path, "a");
    if (!fp) return fail(SRJ_EHIP, std::string("cannot append to the tune cache ") + path);
    const int n = std::fprintf(fp, "%s %s %d %d %.6g\n", kTuneTag, key.c_str(), ti.fused_sweeps, ti.seg_rows,
                               ti.us_per_sweep);
    const bool closed = std::fclose(fp) == 0;
    if (n <= 0 || !closed) return fail(SRJ_EHIP, std::string("cannot append to the tune cache ") + path);
    return SRJ_OK;
}

srj_status srj_plan_poison(srj_plan_t p)
{
    if (!p) return fail(SRJ_EINVAL, "null plan");
    const size_t lo = p->field_elems * fmt_size(p->fmt), hi = p->field_elems * sizeof(double);
    const struct {
        void* ptr;
        size_t bytes;
    } bufs[] = {{p->A.alloc, lo},
                {p->B.alloc, lo},
                {p->blo.alloc, lo},
                {p->b64f.alloc, hi},
                {p->x64.alloc, hi},
                {p->partials, sizeof(double) * 2 * (size_t)residual_blocks(p->geo)}};
    for (const auto& b : bufs)
        if (b.ptr) HIPCHK(hipMemsetAsync(b.ptr, 0xFF, b.bytes, p->stream));
    HIPCHK(hipStreamSynchronize(p->stream));
    return SRJ_OK;
}

srj_status srj_solve_ex(srj_plan_t p, double* u, const double* f, srj_solve_opts* opts, srj_solve_info* info)
{
    fill_info(info, 0, 0, NAN, 0, SRJ_EINVAL);
    if (!p || !u || !f || !opts) return fail(SRJ_EINVAL, "null argument");
    opts->history_len = 0;
    if (!(opts->tol >= 0) || opts->max_sweeps < 0) return fail(SRJ_EINVAL, "bad tolerance or sweep budget");
    if (opts->start_offset < 0 || opts->start_offset >= p->M)
        return fail(SRJ_EINVAL, "start_offset must be in [0, M)");
    if (opts->history_cap < 0 || (opts->history_cap > 0 && !opts->history))
        return fail(SRJ_EINVAL, "history needs a buffer of history_cap entries");
    HIPCHK(hipEventRecord(p->ev0, p->stream));
    HIPCHK(launch_copy_in(p->fmt, u, p->A.origin, p->geo, p->stream));
    HIPCHK(launch_copy_in(p->fmt, u, p->B.origin, p->geo, p->stream));
    HIPCHK(load_rhs(p, f));
    DField* cur = nullptr;
    int64_t k = 0, cycles = 0;
    double rr = 0;
    srj_status result;
    History hist;
    hist.out = opts->history;
    hist.cap = opts->history_cap;
    srj_status st = solve_fields(p, opts->tol, opts->max_sweeps, &cur, &k, &cycles, &rr, &result,
                                 opts->start_offset, opts->history ? &hist : nullptr);
    if (st != SRJ_OK) return st;
    opts->history_len = hist.len;
    if (result != SRJ_EDIVERGED) HIPCHK(launch_copy_out(p->fmt, cur->origin, u, p->geo, p->stream));
    return finish_info(p, info, k, cycles, rr, result);
}

srj_status srj_solve(srj_plan_t p, double* u, const double* f, double tol, int64_t max_sweeps,
                     srj_solve_info* info)
{
    fill_info(info, 0, 0, NAN, 0, SRJ_EINVAL);
    if (!p || !u || !f) return fail(SRJ_EINVAL, "null argument");
    if (!(tol >= 0) || max_sweeps < 0) return fail(SRJ_EINVAL, "bad tolerance or sweep budget");
    HIPCHK(hipEventRecord(p->ev0, p->stream));
    HIPCHK(launch_copy_in(p->fmt, u, p->A.origin, p->geo, p->stream));
    HIPCHK(launch_copy_in(p->fmt, u, p->B.origin, p->geo, p->stream));
    HIPCHK(load_rhs(p, f));
    DField* cur = nullptr;
    int64_t k = 0, cycles = 0;
    double rr = 0;
    srj_status result;
    srj_status st = solve_fields(p, tol, max_sweeps, &cur, &k, &cycles, &rr, &result);
    if (st != SRJ_OK) return st;
    if (result != SRJ_EDIVERGED) HIPCHK(launch_copy_out(p->fmt, cur->origin, u, p->geo, p->stream));
    return finish_info(p, info, k, cycles, rr, result);
}

srj_status srj_adjoint(srj_plan_t p, const double* grad_u, double tol, int64_t max_sweeps, double* df,
                       double* dg, srj_solve_info* info)
{
    fill_info(info, 0, 0, NAN, 0, SRJ_EINVAL);
    if (!p || !grad_u) return fail(SRJ_EINVAL, "null argument");
    if (p->fmt != FMT_F64) return fail(SRJ_EINVAL, "the adjoint solve needs an FP64 plan");
    if (p->geo.bc != 0 || p->geo.op) return fail(SRJ_EINVAL, "the adjoint solve needs the Dirichlet Poisson operator");
    if (!(tol >= 0) || max_sweeps < 0) return fail(SRJ_EINVAL, "bad tolerance or sweep budget");
    HIPCHK(hipEventRecord(p->ev0, p->stream));
    HIPCHK(launch_zero(p->fmt, p->A.origin, p->geo, p->stream));
    HIPCHK(launch_zero(p->fmt, p->B.origin, p->geo, p->stream));
    // right-hand side taken as given: b = 1.0 * grad_u exactly
    HIPCHK(launch_rhs(p->fmt, grad_u, 1.0, p->blo.origin, p->b64, p->geo, p->stream));
    DField* cur = nullptr;
    int64_t k = 0, cycles = 0;
    double rr = 0;
    srj_status result;
    srj_status st = solve_fields(p, tol, max_sweeps, &cur, &k, &cycles, &rr, &result);
    if (st != SRJ_OK) return st;
    if (result != SRJ_EDIVERGED && (df || dg))
        HIPCHK(launch_adjoint_out((const double*)cur->origin, grad_u, p->hh, df, dg, p->geo,
                                  p->stream));
    return finish_info(p, info, k, cycles, rr, result);
}

srj_status srj_solve_ir(srj_plan_t p, double* u, const double* f, double tol, int32_t inner_cycles,
                        int32_t max_outer, srj_solve_info* info)
{
    fill_info(info, 0, 0, NAN, 0, SRJ_EINVAL);
    if (!p || !u || !f) return fail(SRJ_EINVAL, "null argument");
    if (!(tol >= 0) || inner_cycles < 1 || max_outer < 0) return fail(SRJ_EINVAL, "bad IR parameters");
    if (p->geo.bc != 0 || p->geo.op) return fail(SRJ_EINVAL, "refinement needs the Dirichlet Poisson operator");
    const double hh = p->hh;
    srj_status st;
    // the binary64 iterate lives in the plan's x64 field, b in b64; A/B hold the correction d
    // and blo the inner right-hand side (the residual in the sweep format)
    DField& u64 = p->x64;
    HIPCHK(hipEventRecord(p->ev0, p->stream));
    HIPCHK(launch_copy_in(FMT_F64, u, u64.origin, p->geo, p->stream));
    HIPCHK(launch_rhs(FMT_F64, f, hh, nullptr, p->b64, p->geo, p->stream));
    double bt2, bmax;
    if ((st = residual_now(p, u64.origin, FMT_F64, 1, &bt2, &bmax)) != SRJ_OK) return st;
    srj_status result = SRJ_OK;
    double rr = 0.0;
    int64_t sweeps = 0;
    int outer = 0;
    if (!is_finite(bt2)) {
        result = SRJ_EDIVERGED;
        rr = NAN;
    } else if (bt2 == 0.0) {
        HIPCHK(launch_zero(FMT_F64, u64.origin, p->geo, p->stream));
    } else {
        for (;;) {
            HIPCHK(launch_residual_to_lo(p->fmt, (const double*)u64.origin, p->b64, p->blo.origin, p->geo,
                                         p->partials, p->dres, p->stream));
            HIPCHK(hipMemcpyAsync(p->hres, p->dres, 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
            HIPCHK(hipStreamSynchronize(p->stream));
            rr = std::sqrt(p->hres[0]) / std::sqrt(bt2);
            if (!is_finite(rr)) {
                result = SRJ_EDIVERGED;
                break;
            }
            if (rr <= tol) break;
            if (outer >= max_outer) {
                result = SRJ_ENOCONV;
                break;
            }
            HIPCHK(launch_zero(p->fmt, p->A.origin, p->geo, p->stream));
            HIPCHK(launch_zero(p->fmt, p->B.origin, p->geo, p->stream));
            DField *cur = &p->A, *nxt = &p->B;
            if ((st = run_sweeps(p, &cur, &nxt, p->blo.origin, 0, (int64_t)inner_cycles * p->M)) != SRJ_OK)
                return st;
            sweeps += (int64_t)inner_cycles * p->M;
            HIPCHK(launch_update(p->fmt, (double*)u64.origin, cur->origin, p->geo, p->stream));
            outer += 1;
        }
    }
    if (result != SRJ_EDIVERGED) HIPCHK(launch_copy_out(FMT_F64, u64.origin, u, p->geo, p->stream));
    HIPCHK(hipEventRecord(p->ev1, p->stream));
    HIPCHK(hipEventSynchronize(p->ev1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, p->ev0, p->ev1));
    fill_info(info, sweeps, outer, rr, ms * 1e-3, result);
    if (result == SRJ_ENOCONV) return fail(result, "tolerance not reached within max_outer");
    if (result == SRJ_EDIVERGED) return fail(result, "non-finite residual");
    return SRJ_OK;
}

srj_status srj_schedule_optimal(int32_t P, double kappa_min, double kappa_max, double* omega, double* beta,
                                int64_t* q, double* kappa)
{
    if (!omega || !beta || !q) return fail(SRJ_EINVAL, "null argument");
    Optimum o;
    std::string err;
    if (!optimal_schedule(P, kappa_min, kappa_max, &o, &err)) return fail(SRJ_ESCHEDULE, err);
    std::vector<int64_t> qq = floor_counts(o.beta);
    for (int i = 0; i < P; ++i) {
        omega[i] = o.w[i];
        beta[i] = o.beta[i];
        q[i] = qq[i];
    }
    if (kappa)
        for (int j = 0; j + 1 < P; ++j) kappa[j] = o.kappa[j];
    return SRJ_OK;
}

srj_status srj_schedule_counts(int32_t P, const double* beta, const double* omega, double kappa_min,
                               double kappa_max, int32_t q_rounding, int64_t* q)
{
    if (!beta || !q) return fail(SRJ_EINVAL, "null argument");
    if (P < 1 || P > SRJ_MAX_LEVELS) return fail(SRJ_EINVAL, "P must be in [1, 16]");
    if (q_rounding < 0 || q_rounding > 3) return fail(SRJ_EINVAL, "q_rounding must be 0, 1, 2 or 3");
    if (q_rounding == 3 && (!omega || P > 12 || !(kappa_min > 0) || !(kappa_max > kappa_min)))
        return fail(SRJ_EINVAL, "q_rounding 3 needs weights, P <= 12 and 0 < kappa_min < kappa_max");
    for (int i = 0; i < P; ++i)
        if (!(beta[i] > 0) || !std::isfinite(beta[i])) return fail(SRJ_EINVAL, "fractions must be positive");
    std::vector<int64_t> qq = round_counts(std::vector<double>(beta, beta + P), q_rounding, omega, kappa_min, kappa_max);
    if ((int)qq.size() != P) return fail(SRJ_EINVAL, "integer counts could not be formed");
    std::memcpy(q, qq.data(), sizeof(int64_t) * (size_t)P);
    return SRJ_OK;
}

srj_status srj_schedule_order(int32_t P, const double* omega, const int64_t* q, double kappa_min,
                              double kappa_max, int32_t ordering, int32_t* seq)
{
    if (!omega || !q || !seq) return fail(SRJ_EINVAL, "null argument");
    if (P < 1 || P > SRJ_MAX_LEVELS) return fail(SRJ_EINVAL, "P must be in [1, 16]");
    if (ordering != 0 && ordering != 1) return fail(SRJ_EINVAL, "ordering must be 0 or 1");
    if (!(kappa_min > 0) || !(kappa_max > kappa_min)) return fail(SRJ_EINVAL, "bad interval");
    std::vector<int32_t> s = order_steps(P, omega, q, kappa_min, kappa_max, ordering);
    std::memcpy(seq, s.data(), sizeof(int32_t) * s.size());
    return SRJ_OK;
}

}  // extern "C"
