// Launchers of the SRJ device kernels (gfx950).  All pointers are device pointers to
// padded fields: element (k, i, j) of a field lives at origin[(k * py + i) * px + j], with
// i, j, k running over 0..n+1 (ring included), px the row pitch and py = ny + 2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace srj {

enum Fmt { FMT_F64 = 0, FMT_F32 = 1, FMT_BF16 = 2 };

constexpr int kMaxFuse = 10;   // largest number of sweeps fused into one 2D launch
constexpr int kMaxFuse3d = 5;  // largest number of sweeps fused into one 3D launch

struct Geo {
    int ndim;
    int64_t nx, ny, nz;  // interior sizes (nz = 1 in 2D)
    int64_t px, py;      // row pitch (elements) and rows per plane (ny + 2)
    // operator weights, the equation multiplied through by h_x^2: 1 on the x neighbours,
    // wy = h_x^2 / h_y^2, wz = h_x^2 / h_z^2 (1 in 2D), diagonal dg = 2 (1 + wy) in 2D and
    // 2 ((1 + wy) + wz) in 3D; equal spacings give 1, 1 and 2d
    double wy, wz, dg;
    // boundary: 0 Dirichlet (the ring holds the data), 1 homogeneous Neumann (cell-centred:
    // a neighbour across the boundary is the cell itself; the ring is never read)
    int bc;
    // variable-coefficient operator (op = 1): Jacobi-scaled neighbour weights a_nb / a_P as
    // padded fields w[0..2d) (W, E, S, N[, D, U]) and an optional mask field (nonzero: a
    // fixed point); the step is u' = u + w_k ((s + b) - u) with s the weighted neighbour sum
    int op;
    const double* w[6];
    const uint8_t* mask;
};

// Geo's operator weights for spacings h[0..ndim); iso is set when they are all equal.
inline void geo_set_weights(Geo& g, const double* h, bool* iso)
{
    const double hxx = h[0] * h[0];
    g.wy = hxx / (h[1] * h[1]);
    g.wz = g.ndim == 3 ? hxx / (h[2] * h[2]) : 1.0;
    g.dg = g.ndim == 2 ? 2.0 * (1.0 + g.wy) : 2.0 * ((1.0 + g.wy) + g.wz);
    if (iso) *iso = g.wy == 1.0 && g.wz == 1.0;
}

struct Coefs {
    double c[kMaxFuse];  // c = w / (2d) of consecutive sweeps
};

size_t fmt_size(Fmt f);

// user (dense FP64, ring included) -> field in format f (all points, ring included)
hipError_t launch_copy_in(Fmt f, const double* user, void* field, const Geo& g, hipStream_t s);
// field -> user interior (ring of user untouched)
hipError_t launch_copy_out(Fmt f, const void* field, double* user, const Geo& g, hipStream_t s);
// b = (h*h) * f on the interior: blo in format f (may be null), b64 in FP64 (may be null)
hipError_t launch_rhs(Fmt f, const double* user_f, double hh, void* blo, double* b64, const Geo& g,
                      hipStream_t s);
// One sweep in -> out with coefficient c = w / g.dg (2D or 3D), with the operator weights of g.
hipError_t launch_sweep_unfused(Fmt f, const void* in, void* out, const void* b, const Geo& g,
                                double c, hipStream_t s);
// T consecutive 2D sweeps in -> out in one launch with coefficients co.c[0..T), row
// segments of H output rows per wave.  flip (0 or 1) reverses the direction every segment
// streams in; callers alternate it from launch to launch (it changes no result).  nt: binary64
// stores carry the non-temporal hint (ignored for the other formats; it changes no result).
// (The temporally blocked kernels implement the equal-spacing Dirichlet operator only.)
hipError_t launch_sweep_fused(Fmt f, const void* in, void* out, const void* b, const Geo& g,
                              const Coefs& co, int T, int H, int flip, bool nt, hipStream_t s);
// T <= lds_fuse_max() (8) binary64 sweeps of a 2D grid with unequal spacings, Neumann
// boundaries or a point-wise operator in one launch, on tiles held in LDS with T-wide halos
// (sweep2d_lds.hip).  lds_fuse_fits: 2D binary64.
int lds_fuse_max();
bool lds_fuse_fits(const Geo& g, Fmt f);
hipError_t launch_sweep_lds2d(const void* in, void* out, const void* b, const Geo& g, const Coefs& co, int T,
                              hipStream_t s);

// T <= kMaxFuse3d sweeps (coefficients co.c[0..T)) of a 3D grid in one launch: x-y tiles of
// 64 x 30 or 64 x 32 with T-wide halos, streamed in z, upwards or (flip = 1) downwards;
// callers alternate flip from launch to launch (it changes no result).  Needs
// fused3d_fits(g, f): a padded z plane below 1 GiB (its stores are addressed within one plane).
inline bool fused3d_fits(const Geo& g, Fmt f)
{
    return g.px * g.py * (int64_t)fmt_size(f) < ((int64_t)1 << 30) - 4096;
}
hipError_t launch_sweep_fused3d(Fmt f, const void* in, void* out, const void* b, const Geo& g,
                                const Coefs& co, int T, int flip, hipStream_t s);
// Default sweeps per fused 3D launch for a grid (5, 4 or 3): the depth whose launch shape a
// cost model of the tiling (rounds of blocks, steps per block) gives the lowest time per sweep.
int fused3d_default_depth(const Geo& g, Fmt f);
// sum r^2 and max |r| of r = b64 - A u (binary64); zero_interior treats u's interior as 0.
// partials must hold 2 * residual_blocks(g) doubles; result receives {sum, max}.
int residual_blocks(const Geo& g);
// One binary64 sweep u -> out with coefficient c fused with the residual norms of u: the
// (sum r^2, max |r|) pair lands in result[0..1] as launch_residual would put it there.
hipError_t launch_sweep_residual(const double* u, double* out, const double* b64, const Geo& g, double c,
                                 double* partials, double* result, hipStream_t s);
hipError_t launch_residual(Fmt f, const void* u, const double* b64, const Geo& g, int zero_interior,
                           double* partials, double* result, hipStream_t s);
// IR: r = b64 - A u64 (binary64) written to rlo in format f, with its norms (as above).
hipError_t launch_residual_to_lo(Fmt f, const double* u64, const double* b64, void* rlo,
                                 const Geo& g, double* partials, double* result, hipStream_t s);
// r = b64 - A u64 (binary64) into a user array (dense layout, ring included, ring set to 0)
hipError_t launch_residual_out(const double* u64, const double* b64, double* r_user, const Geo& g, hipStream_t s);
// IR: u64 interior += widen(d)
hipError_t launch_update(Fmt f, double* u64, const void* d, const Geo& g, hipStream_t s);
// adjoint outputs from the FP64 field lam: user df = hh * lam (interior, ring 0) and user
// dg = grad_u + lam at the interior neighbour, on each ring cell (interior 0); df or dg may
// be null
hipError_t launch_adjoint_out(const double* lam, const double* grad_u, double hh, double* df, double* dg,
                              const Geo& g, hipStream_t s);
// Variable-coefficient operator: from the user's coefficient arrays coef (2d + 1 consecutive
// full-grid arrays a_P, a_W, a_E, a_S, a_N[, a_D, a_U]) write the scaled weights
// w[k] = a_{k+1} / a_P and a_P itself into padded fields (interior points; 0 on the ring),
// and the user's mask (may be null) into a padded uint8 field.
hipError_t launch_op_setup(const double* coef, const uint8_t* mask_user, double* const* w, double* ap,
                           uint8_t* mask, const Geo& g, hipStream_t s);
// b = f / a_P at the free interior points (0 elsewhere), into b64 (padded, binary64)
hipError_t launch_op_rhs(const double* user_f, const double* ap, double* b64, const Geo& g, hipStream_t s);
// Whole solves of small 2D grids in one workgroup with the grid in LDS (binary64 Dirichlet
// Poisson plans of at most kSmallPoints points including the ring): iterate pair and source
// in LDS, residual checks at k = 0 and every cycle end, as srj_solve.  in/b/out are padded
// fields, cseq the M coefficients of a cycle (device), res receives {sweeps, cycles, relres,
// status} (device, 4 doubles).
constexpr int kSmallPoints = 6656;
bool small_solve_fits(const Geo& g);
hipError_t launch_small_solve(const double* in, const double* b, double* out, const Geo& g, const double* cseq,
                              int64_t M, double tol, int64_t max_sweeps, double* res, hipStream_t s);
// set every element of the field (ring included) to zero with a fill kernel
hipError_t launch_zero(Fmt f, void* field, const Geo& g, hipStream_t s);

}  // namespace srj
