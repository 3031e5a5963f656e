/*
 * libsrj -- Scheduled Relaxation Jacobi (SRJ) solver for the finite-difference Poisson
 * problem on one AMD Instinct MI355X (gfx950).  C ABI.
 *
 * Method: Adsuara, Cordero-Carrion, Cerda-Duran, Aloy, "Scheduled Relaxation Jacobi
 * method: improvements and applications".  Sec. 2 defines the scheme (P weights
 * w_1 > ... > w_P, weight i applied q_i times per cycle of M = sum q_i steps, cycles
 * repeated); Sec. 3.1 (Eq. 2nd-order_CD) the weighted-Jacobi step; Sec. 3 the optimal
 * weights; Sec. 4.3 the integer counts; Sec. 5.1 the Dirichlet Poisson setting and the
 * need to spread the large weights over the cycle.
 *
 * Problem solved:  -lap(u) = f  on a box of n_i interior points per axis with spacing h_i
 * on axis i and Dirichlet data on the ring of points around the box (Sec. 5.1).  The
 * equation is multiplied through by h_x^2: weight 1 on the x neighbours, wy = h_x^2/h_y^2,
 * wz = h_x^2/h_z^2 on the others, diagonal dg = 2(1 + wy) in 2D, 2((1 + wy) + wz) in 3D
 * (2d when the spacings are equal).  With b = (h_x*h_x) f, one step with weight w
 * (c = w / dg) is
 *     u' = u + c * ( ((W+E) + wy (S+N) [+ wz (D+U)] + b) - dg u ),
 * evaluated in that association, then + b, then - dg u, then u + c*t, each operation
 * rounded on its own (with equal spacings the kernels form "- 4u" in 2D with a fused
 * multiply-add, which is the same value since 4u is exact).  The residual r = b - A u
 * (A = dg I minus the weighted neighbour sum) is the t of that step;
 * relres = ||r||_2 / ||b~||_2, b~ being the residual of the state with a zero interior
 * (source plus boundary terms).  Plans with unequal spacings fuse sweeps only in 2D binary64
 * (on tiles held in LDS, see srj_plan_set_fusion); otherwise they run one sweep per launch.
 *
 * Array layout at the ABI: dense, row-major, x fastest, ring included:
 *   2D: (n[1] + 2) rows of (n[0] + 2) doubles;  3D: (n[2]+2) x (n[1]+2) x (n[0]+2).
 * u and f are DEVICE pointers to binary64 arrays owned by the caller.  u is in/out:
 * its ring holds the Dirichlet values (never written), its interior the initial guess on
 * entry and the result on return.  f's ring is ignored.
 *
 * Errors: every call returns an srj_status; no exception crosses the ABI.
 * srj_last_error() returns a thread-local message for the last failing call.
 * Streams: all device work runs on the plan's stream (a hipStream_t passed as void*,
 * NULL = default stream).  One plan must not be used from two host threads at once.
 */
#ifndef SRJ_H
#define SRJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SRJ_MAX_LEVELS 16

typedef enum {
    SRJ_OK = 0,
    SRJ_EINVAL = 1,     /* bad argument: null pointer, n < 1, ndim not 2/3, bad schedule */
    SRJ_ENOMEM = 2,     /* device or host allocation failed */
    SRJ_EHIP = 3,       /* a HIP runtime call failed */
    SRJ_ESCHEDULE = 4,  /* optimiser did not converge, or the integer scheme has Gamma_q >= 1 */
    SRJ_ENOCONV = 5,    /* tolerance not reached within the sweep / outer budget */
    SRJ_EDIVERGED = 6   /* residual became inf or NaN */
} srj_status;

/* Storage format of the iterate during sweeps.  SRJ_F64 computes in binary64;
 * SRJ_F32 stores and computes in binary32; SRJ_BF16 stores bfloat16 (round to nearest
 * even on every store) and computes in binary32.  Residual norms are always binary64. */
typedef enum { SRJ_F64 = 0, SRJ_F32 = 1, SRJ_BF16 = 2 } srj_dtype;

typedef struct {
    int32_t ndim;     /* 2 or 3 */
    int64_t n[3];     /* interior points per axis, n[0] = x (fastest); n[2] unused in 2D */
    double h[3];      /* spacing per axis, h[0] = x (unit box: 1 / (n_i + 1)); h[2] unused in 2D */
    int32_t dtype;    /* srj_dtype of the sweeps */
    int32_t bc;       /* 0: Dirichlet, the ring holds the boundary values.  1: homogeneous
                         Neumann on a cell-centred grid of n_i >= 2 cells per axis (Sec. 3.1,
                         Eq. Laplace; unit box: h_i = 1 / n_i): the ring is a row of ghost
                         cells mirroring their neighbours and is never read, a neighbour
                         across the boundary being the cell itself.  Neumann plans are binary64;
                         in 2D they fuse up to 8 sweeps per launch on tiles held in LDS, in
                         3D they run one sweep per launch; the operator is singular (constants
                         solve A u = 0), so the source must have zero mean and srj_solve
                         measures relres against the initial residual ||r(u_0)|| (u_0
                         returned unchanged if that is 0).  The schedule's default
                         interval starts at the smallest nonzero symbol, (2/d) sin^2(pi / 2N)
                         with N = max n_i for equal spacings (Eq. boundaries1D3D).  Not for
                         srj_solve_ir, srj_adjoint, batches or srj_residual_static. */
} srj_grid;

/* Schedule request (Sec. 2-4).
 *  omega == NULL: optimise P levels (Sec. 3) on [kappa_min, 2] (Eq. boundaries).
 *    The lower end: kappa_min > 0 as given; else n_eff > 0 takes the Neumann table row of
 *    resolution N = n_eff, sin^2(pi / (2 N)) (Eq. boundaries; e.g. the rows N = 550 and
 *    N = 250 of Sec. 5.1); else (both 0) the exact smallest Jacobi symbol of the grid,
 *    (2/d) sum_i sin^2(pi / (2 (n_i + 1))) with equal spacings (Eq. effectiveNDirichlet with
 *    N_i = n_i + 1 zones), 4 (s_x + wy s_y [+ wz s_z]) / dg otherwise.  Giving both is an error.
 *    Counts from the fractions (Sec. 4.3), q_rounding: 0 floor(beta_i / beta_1) (the
 *    paper's choice), 1 nearest integer, 2 ceiling, 3 floor or ceiling per level, whichever
 *    combination has the smallest per-step factor max |prod (1 - w_i k)^q_i|^(1/M) over
 *    [kappa_min, 2] (P <= 12; exact ties to fewer ceilings, then to the earlier combination
 *    in binary order with level 2 the lowest bit).  q_1 = 1 in every mode.
 *  omega != NULL: P explicit weights, strictly descending, with P counts q >= 1 (n_eff and
 *    kappa_min then only set the interval the order is built on; q_rounding is ignored).
 *  ordering: 0 balanced greedy order of the M steps (default), 1 even spread of each
 *    weight over the cycle (Sec. 5.1), 2 explicit: sequence[0..M) of level indices. */
typedef struct {
    int32_t P;
    const double* omega;
    const int64_t* q;
    double kappa_min;
    double n_eff;
    int32_t q_rounding;
    int32_t ordering;
    const int32_t* sequence;
    int64_t M;
} srj_schedule;

/* Description of a plan's schedule (srj_plan_describe). */
typedef struct {
    int32_t P;
    int64_t M;
    double omega[SRJ_MAX_LEVELS];
    double beta[SRJ_MAX_LEVELS];   /* real fractions (0 for explicit schedules) */
    int64_t q[SRJ_MAX_LEVELS];
    double kappa_min, kappa_max;   /* interval the scheme was checked on */
    double rho;                    /* sum w_i beta_i (Eq. rho); with integer q: sum w_i q_i / M */
    double gamma_q_max;            /* max over [kappa_min, kappa_max] of |prod (1-w_i k)^q_i|^(1/M) */
    double prefix_peak_log10;      /* largest partial product of the ordered cycle, log10 */
    double suffix_peak_log10;
    int32_t fused_sweeps;          /* sweeps fused per launch by the 2D/3D kernels */
    int32_t resident;              /* 1: srj_solve runs in one workgroup with the grid in LDS */
    int32_t store_nt;              /* 1: the register-streamed fused 2D binary64 launches
                                      (equal spacings, Dirichlet) store with the non-temporal
                                      cache hint: grids whose input, output and b fields
                                      exceed the 256 MiB memory-side cache but fit in twice it */
} srj_plan_desc;

typedef struct {
    int64_t sweeps;   /* weighted-Jacobi sweeps applied */
    int64_t cycles;   /* completed M-cycles (IR: outer steps) */
    double relres;    /* relres of the returned state */
    double seconds;   /* device time between the first and the last kernel of the call */
    int32_t status;
} srj_solve_info;

typedef struct srj_plan_s* srj_plan_t;

/* Create a plan: validates the grid, builds the schedule and its coefficient sequence
 * c_k = w_k / dg, allocates the plan-owned device buffers (two iterate buffers in the sweep
 * format, the scaled source in the sweep format and in binary64, a binary64 iterate for
 * refinement and residual evaluation, reduction scratch): solves, sweeps, residuals and
 * refinement then allocate nothing.  Returns SRJ_ESCHEDULE if the optimiser fails or the
 * integer scheme is not convergent on the grid's spectrum. */
srj_status srj_plan(const srj_grid* grid, const srj_schedule* schedule, void* stream,
                    srj_plan_t* out);
void srj_plan_destroy(srj_plan_t plan);
srj_status srj_plan_describe(srj_plan_t plan, srj_plan_desc* out);
/* Copy the ordered level indices of one cycle (cap >= M) into seq. */
srj_status srj_plan_sequence(srj_plan_t plan, int32_t* seq, int64_t cap);
/* Small binary64 2D Dirichlet grids (at most 6656 points with the ring, e.g. 79 x 79 interior)
 * are solved by srj_solve in one launch of one workgroup holding the grid in LDS (resident = 1
 * in srj_plan_desc); srj_plan_set_fusion turns that off.
 * Override the number of sweeps fused per launch (0 = unfused reference kernel; at most
 * 10 in 2D, 5 in 3D; the default is 10 in 2D and, in 3D, 5, 4 or 3, whichever a model of the
 * launch shape (blocks against compute units, steps per block) gives the lowest time per
 * sweep; 2D binary64
 * plans with unequal spacings, Neumann boundaries or an operator fuse at most 8, on tiles held
 * in LDS, 8 by default; in 3D, and in binary32 / bfloat16, such plans sweep once per launch)
 * and the output rows each wave of the fused 2D kernel computes (seg_rows = 0, the
 * default: chosen per launch so that the grid of waves fills the device's resident wave
 * slots once, from the kernel's occupancy and the number of compute units).  The results
 * do not depend on either value. */
srj_status srj_plan_set_fusion(srj_plan_t plan, int32_t fused_sweeps, int32_t seg_rows);

/* Solve to ||r||_2 / ||b~||_2 <= tol, checked at sweep 0 and at every cycle end (every
 * sweep for M = 1).  Stops with SRJ_ENOCONV when the next cycle would exceed max_sweeps
 * (u then holds the last checked state), SRJ_EDIVERGED on a non-finite residual (u
 * unspecified).  Synchronises with the host once per check. */
srj_status srj_solve(srj_plan_t plan, double* u, const double* f, double tol, int64_t max_sweeps,
                     srj_solve_info* info);

/* Options of srj_solve_ex; zero-initialise, then set what is used. */
typedef struct {
    double tol;             /* as srj_solve */
    int64_t max_sweeps;     /* sweeps this call may apply */
    int64_t start_offset;   /* 0 <= start_offset < M: u is the iterate after start_offset sweeps
                               of a cycle (a checkpoint taken mid-cycle, e.g. after srj_sweeps);
                               the solve first applies the cycle's remaining M - start_offset
                               sweeps and checks at that cycle end */
    double* history;        /* host array or NULL: relres of every check, in order */
    int64_t history_cap;    /* entries history holds (the first history_cap checks are kept) */
    int64_t history_len;    /* out: checks made (can exceed history_cap); 0 if history is NULL */
} srj_solve_opts;

/* srj_solve with a start offset and a record of the residual at every check (the history
 * the paper plots against sweeps, Sec. 4, and the state a resumed solve needs: u and the
 * step index k mod M).  A solve resumed from the iterate after k_c sweeps of an interrupted
 * solve, with start_offset = k_c mod M, applies the same sweeps, stops at the same sweep
 * (counted from k_c) and returns the same bits as the uninterrupted one, provided that one
 * had not stopped before k_c.  With Neumann boundaries the reference of relres is the
 * residual of the state passed in.  If the budget does not reach the end of the started
 * cycle, u is returned unchanged with SRJ_ENOCONV, 0 sweeps and the relres of u.
 * A solve with a history or a start offset runs the multi-launch path even on a plan that
 * srj_solve would solve in LDS (same results).  Other arguments and status as srj_solve. */
srj_status srj_solve_ex(srj_plan_t plan, double* u, const double* f, srj_solve_opts* opts,
                        srj_solve_info* info);

/* Apply exactly nsweeps scheduled sweeps to u, the first one being step k0 (mod M) of the
 * cycle.  No convergence checks.  If stats is not NULL, stats[0] receives the device time
 * in seconds of the sweep launches alone (HIP events on the plan's stream around them) and
 * stats[1] the number of kernel launches they took. */
srj_status srj_sweeps(srj_plan_t plan, double* u, const double* f, int64_t k0, int64_t nsweeps,
                      double* stats);

/* norms[0] = ||r||_2, norms[1] = max |r|, norms[2] = ||b~||_2, norms[3] = relres, for
 * r = b - A u in binary64.  r_out (device, full-grid layout, ring set to 0) may be NULL.
 * (Neumann grids: b~ = b, the residual of the zero state.) */
srj_status srj_residual(srj_plan_t plan, const double* u, const double* f, double* r_out,
                        double norms[4]);

/* A plan for a variable-coefficient operator given point by point (Sec. 5.3's Grad-Shafranov
 * operator with its C^2 Psi term and masked region, Sec. 5.2's variable-coefficient stencils):
 *     (A u)_P = a_P u_P - sum over the 2d neighbours of a_nb u_nb = f_P
 * at every interior point whose mask is 0; the ring and masked points hold fixed values.
 * coef: DEVICE, 2d + 1 consecutive arrays of the full-grid ABI layout, a_P, a_W, a_E, a_S,
 * a_N (, a_D, a_U) -- W/E along x, S/N along y, D/U along z -- read once here (a_P nonzero at
 * the free points).  mask: DEVICE uint8 array of the same layout (nonzero = fixed point), or
 * NULL.  The operator is Jacobi-scaled once, w_nb = a_nb / a_P and b = f / a_P (one IEEE
 * division each), and one step with weight w is
 *     s = (w_W W + w_E E) + (w_S S + w_N N) [+ (w_D D + w_U U)];  t = (s + b) - u;  u' = u + w t,
 * evaluated in that association; relres is the same Jacobi-scaled residual t measured against
 * t of the state whose free points are zero.  grid->h is ignored (the coefficients carry the
 * scaling), grid->dtype must be SRJ_F64 and grid->bc 0.  The schedule must be explicit or give
 * kappa_min or n_eff (the operator's spectrum is not known to the library).  In 2D such plans
 * fuse up to 8 sweeps per launch on 32 x 32 tiles held in LDS with their weights and mask, in
 * 3D they run one sweep per launch; they serve srj_solve, srj_sweeps and srj_residual (norms
 * of t); not srj_solve_ir or srj_adjoint. */
srj_status srj_plan_operator(const srj_grid* grid, const srj_schedule* schedule, const double* coef,
                             const uint8_t* mask, void* stream, srj_plan_t* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the residual norms of srj_residual for a
 * grid described by grid (ndim, n, h; dtype ignored), computed from the caller's DEVICE
 * arrays u and f (ABI layout) without a plan, without allocating and without synchronising:
 * every launch goes on stream (a hipStream_t, NULL = default stream).  norms (DEVICE, 4
 * doubles) receives ||r||_2, max |r|, ||b~||_2, relres when the stream reaches that point;
 * r_out (DEVICE, full layout, may be NULL) receives r with a zero ring.  The results are
 * bit-identical to srj_residual's.  Scratch: a 2 MiB array per GPU held by the library until
 * the process ends (per-block partial sums, fully rewritten by every call), enough for grids
 * of at most 524288 lines (n[1] in 2D, n[1] * n[2] in 3D); larger grids return SRJ_EINVAL
 * before anything is launched.  Calls that overlap on one GPU (two streams, or two threads)
 * race on that array: order them. */
srj_status srj_residual_static(const srj_grid* grid, const double* u, const double* f, double* r_out,
                               double* norms, void* stream);

/* FP64 iterative refinement around the plan's low-precision sweeps (plan dtype F32 or
 * BF16; an F64 plan runs the same loop with binary64 sweeps, its inner right-hand side kept
 * apart from b): repeat { r = b - A u (binary64);
 * stop if relres <= tol; d = inner_cycles SRJ cycles on A d = r from d = 0 with a zero
 * ring, in the plan's format; u += d (binary64) } at most max_outer times. */
srj_status srj_solve_ir(srj_plan_t plan, double* u, const double* f, double tol,
                        int32_t inner_cycles, int32_t max_outer, srj_solve_info* info);

/* Adjoint of srj_solve for a loss L(u) of the solution (the differentiable solve).
 * The forward map is (f, g) -> u with u = g on the ring and A u = b~ inside, where
 * A = 2d I - (interior neighbour sum) is symmetric and b~ = h^2 f + (ring values next to
 * each point) (Sec. 5.1 setting).  Given grad_u = dL/du (device, full layout) this solves
 * A lambda = (interior of grad_u) with the plan's schedule and stopping rule (zero ring,
 * zero start), then writes
 *     df = h_x^2 lambda on the interior, 0 on the ring;
 *     dg = grad_u + (axis weight) * (lambda at the interior neighbour) on each ring cell --
 *          the weight of the axis along which the neighbour reads it (1, wy or wz); the
 *          neighbour term is absent on ring cells no stencil reads (2D corners; 3D edges
 *          and corners) -- and 0 on the interior.
 * df or dg may be NULL.  No forward iterate is needed or stored.  FP64 plans only.
 * Status as srj_solve. */
srj_status srj_adjoint(srj_plan_t plan, const double* grad_u, double tol, int64_t max_sweeps,
                       double* df, double* dg, srj_solve_info* info);

/* Batched solves: many independent 2D grids (sizes, spacings and schedules may all
 * differ; one storage format per batch), each solved by the same FP64 refinement as
 * srj_solve_ir with its own schedule (Sec. 2-4 per problem), all advanced together on
 * the device.  One kernel launch per iteration goes over the tiles of every running
 * problem: tiles of a sweeping problem get up to 10 scheduled sweeps, tiles of a problem
 * that finished an inner solve get u + d and its binary64 residual, and the last tile of a
 * problem decides it.  The iterations are replayed from a captured HIP graph on an
 * internal stream (the plan's stream is synchronised first).  Problems never wait on one
 * another; finished problems drop out of the work list. */
typedef struct srj_batch_s* srj_batch_t;
/* grids[count], schedules[count] as for srj_plan (ndim must be 2 with h[0] == h[1], one
 * dtype for all).  The batch owns all device buffers (about 3 FP64 + 3 sweep-format fields
 * per problem). */
srj_status srj_batch_plan(int32_t count, const srj_grid* grids, const srj_schedule* schedules,
                          void* stream, srj_batch_t* out);
/* u[j], f[j]: device FP64 arrays of problem j in the ABI layout (u in/out).  infos[j] (may be
 * NULL) as srj_solve_ir's; seconds[j] (may be NULL): device time from the start of the
 * iterations to the decision that problem j converged (0 if it did not).  Returns SRJ_OK if
 * every problem converged, else SRJ_EDIVERGED or SRJ_ENOCONV (per-problem status in infos). */
srj_status srj_batch_solve(srj_batch_t batch, double* const* u, const double* const* f, double tol,
                           int32_t inner_cycles, int32_t max_outer, srj_solve_info* infos,
                           double* seconds);
void srj_batch_destroy(srj_batch_t batch);

/* Autotuning of the launch shape (no paper counterpart: the paper's sweeps are scalar
 * loops).  The tuner times candidate configurations on the device, on the plan's or
 * batch's own scratch fields (no user data is read or written), keeps the fastest (the
 * configuration in place unless another is at least 3% faster), and returns what it
 * measured.  Results of later solves are bit-identical whatever is
 * chosen; only their speed changes.  Synchronises the plan's stream; takes milliseconds
 * to about a second for the largest grids.
 *   srj_plan_tune: 2D plans time fusion depths {10, 8, 6, 4} x segment heights {automatic,
 *     24, 32, 48, 64, 96, 128}; 3D plans fusion depths {5, 4, 3, 2, 1, 0}; 2D binary64 plans
 *     with unequal spacings, Neumann boundaries or an operator depths {8, 4, 2, 0}.  Sets the
 *     plan's fusion (as srj_plan_set_fusion would).
 *   srj_batch_tune: times the batch's sweep launch with every problem sweeping, for
 *     largest tile heights {32, 64, 128, 256}, and keeps the fastest as the height the
 *     batch starts from (it still shortens tiles as problems finish). */
typedef struct {
    int32_t fused_sweeps;        /* chosen sweeps per launch (batch: 10) */
    int32_t seg_rows;            /* chosen segment / largest tile height (0 = automatic) */
    int32_t candidates;          /* configurations timed */
    double us_per_sweep;         /* device time per sweep of the whole grid / batch, chosen */
    double us_per_sweep_before;  /* the same for the configuration in place before tuning */
} srj_tune_info;
srj_status srj_plan_tune(srj_plan_t plan, srj_tune_info* info);
srj_status srj_batch_tune(srj_batch_t batch, srj_tune_info* info);
/* srj_plan_tune through an on-disk cache (a text file at path, created if missing, one line
 * per tuned configuration).  The key is the device (architecture name and compute-unit
 * count), ndim, n, the storage format, the boundary kind, equal or unequal spacings,
 * operator plans and the cycle length M (launches end at cycle ends).  On a hit the stored launch shape is applied without timing anything
 * (info->candidates = 0, both times = the stored time); on a miss the plan is tuned and a
 * line is appended.  Entries that the plan could not run are ignored.  SRJ_EINVAL for a
 * null path, SRJ_EHIP if the file cannot be written after tuning (the plan is tuned
 * anyway). */
srj_status srj_plan_tune_cached(srj_plan_t plan, const char* path, srj_tune_info* info);

/* Debugging aid: fill the plan's working buffers (the iterate pair, the right-hand sides in
 * the sweep format and in binary64, the refinement iterate and the reduction partials),
 * padding and alignment slack included, with all-one bytes (a NaN in binary64, binary32 and
 * bfloat16).  Later calls write the points they use before reading them, so a kernel that
 * read outside its stencil's points would turn results into NaN; results must stay
 * bit-identical.  What the plan was built from stays: the schedule's coefficients and an
 * operator plan's weights and mask.  Not for graph capture (it clears with memset). */
srj_status srj_plan_poison(srj_plan_t plan);

/* Host-only schedule computations (no device needed). */
/* Optimal P-level weights/fractions on [kappa_min, kappa_max] (Sec. 3) and counts
 * q_i = floor(beta_i / beta_1) (Sec. 4.3).  kappa (P-1 values, may be NULL) receives the
 * interior maxima of Gamma. */
srj_status srj_schedule_optimal(int32_t P, double kappa_min, double kappa_max, double* omega,
                                double* beta, int64_t* q, double* kappa);
/* Integer counts q[0..P) from fractions beta (Sec. 4.3), rounding mode as srj_schedule's
 * q_rounding (0 floor, 1 nearest, 2 ceiling, 3 best floor/ceiling combination on
 * [kappa_min, kappa_max] for the weights omega, P <= 12; omega may be NULL for modes 0-2). */
srj_status srj_schedule_counts(int32_t P, const double* beta, const double* omega, double kappa_min,
                               double kappa_max, int32_t q_rounding, int64_t* q);
/* Order of the M steps for weights omega / counts q (ordering 0 balanced, 1 even). */
srj_status srj_schedule_order(int32_t P, const double* omega, const int64_t* q, double kappa_min,
                              double kappa_max, int32_t ordering, int32_t* seq);

const char* srj_status_string(srj_status s);
const char* srj_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SRJ_H */
