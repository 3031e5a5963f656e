/*
 * CPU oracle for the Scheduled Relaxation Jacobi (SRJ) hot path -- TEST INFRASTRUCTURE.
 *
 * Plain, slow, obviously correct loops.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library; the product path never does.
 * It shares no code with the HIP library.
 *
 * Discretisation (paper Sec. 3.1, Eq. 2nd-order_CD, written for the Poisson problem
 * of Sec. 5.1 with the sign convention -lap(u) = f):
 *   grid of n_i interior points per dimension, spacing h_x, h_y (, h_z), ring of Dirichlet
 *   values.  Multiplied through by h_x^2 the operator has weight 1 on the x neighbours,
 *   wy = h_x^2 / h_y^2 on the y neighbours, wz = h_x^2 / h_z^2 on the z neighbours and the
 *   diagonal dg = 2 ((1 + wy) + wz) (2 (1 + wy) in 2D); with equal spacings wy = wz = 1 and
 *   dg = 2d.  b = (h_x*h_x) * f ;  weighted Jacobi step with weight w, c = w / dg:
 *     s  = (W + E) + wy (S + N)         [ + wz (D + U) in 3D ]
 *     t  = (s + b) - dg * u             (t is the residual b - A u of the input state)
 *     u' = u + c * t
 *   The weights come in as wt = {wy, wz, dg}.  The association above is fixed; the file is
 *   compiled with -ffp-contract=off so no multiply-add is fused.  With unit weights every
 *   product by a weight is exact and the step is the equal-spacing step.
 *
 * Layout: row-major, x fastest.  2D: (ny+2) rows of (nx+2); 3D: (nz+2) planes of
 * (ny+2) rows of (nx+2).  Index 0 and n+1 of every dimension is the Dirichlet ring.
 */
#include <stdint.h>
#include <string.h>
#include <math.h>

#define I2(i, j) ((size_t)(i) * (size_t)(nx + 2) + (size_t)(j))
#define I3(k, i, j) (((size_t)(k) * (size_t)(ny + 2) + (size_t)(i)) * (size_t)(nx + 2) + (size_t)(j))

/* ---------------------------------------------------------------- FP64 sweeps */

/* One weighted-Jacobi step, 2D 5-point (Eq. 2nd-order_CD).  out's ring is not touched. */
void or_sweep2d(int64_t nx, int64_t ny, const double* u, const double* b, const double* wt, double c,
                double* out)
{
    const double wy = wt[0], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= ny; ++i) {
        for (int64_t j = 1; j <= nx; ++j) {
            double s = (u[I2(i, j - 1)] + u[I2(i, j + 1)]) + wy * (u[I2(i - 1, j)] + u[I2(i + 1, j)]);
            double t = (s + b[I2(i, j)]) - dg * u[I2(i, j)];
            out[I2(i, j)] = u[I2(i, j)] + c * t;
        }
    }
}

/* One weighted-Jacobi step, 3D 7-point (Eq. 2nd-order_CD extended to d = 3, Sec. 3.1). */
void or_sweep3d(int64_t nx, int64_t ny, int64_t nz, const double* u, const double* b, const double* wt,
                double c, double* out)
{
    const double wy = wt[0], wz = wt[1], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k <= nz; ++k) {
        for (int64_t i = 1; i <= ny; ++i) {
            for (int64_t j = 1; j <= nx; ++j) {
                double s = ((u[I3(k, i, j - 1)] + u[I3(k, i, j + 1)]) +
                            wy * (u[I3(k, i - 1, j)] + u[I3(k, i + 1, j)])) +
                           wz * (u[I3(k - 1, i, j)] + u[I3(k + 1, i, j)]);
                double t = (s + b[I3(k, i, j)]) - dg * u[I3(k, i, j)];
                out[I3(k, i, j)] = u[I3(k, i, j)] + c * t;
            }
        }
    }
}

/* Plain Jacobi written from its own definition: u' = (sum of neighbours + b) / (2d).
 * Kept separate from the weighted step so that "w = 1 is Jacobi" is a real check. */
void or_jacobi2d(int64_t nx, int64_t ny, const double* u, const double* b, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= ny; ++i)
        for (int64_t j = 1; j <= nx; ++j)
            out[I2(i, j)] = (u[I2(i, j - 1)] + u[I2(i, j + 1)] + u[I2(i - 1, j)] + u[I2(i + 1, j)] +
                             b[I2(i, j)]) / 4.0;
}

void or_jacobi3d(int64_t nx, int64_t ny, int64_t nz, const double* u, const double* b, double* out)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k <= nz; ++k)
        for (int64_t i = 1; i <= ny; ++i)
            for (int64_t j = 1; j <= nx; ++j)
                out[I3(k, i, j)] = (u[I3(k, i, j - 1)] + u[I3(k, i, j + 1)] + u[I3(k, i - 1, j)] +
                                    u[I3(k, i + 1, j)] + u[I3(k - 1, i, j)] + u[I3(k + 1, i, j)] +
                                    b[I3(k, i, j)]) / 6.0;
}

/* Run `nsweeps` scheduled steps: step s uses c_seq[(k0 + s) mod M] (Sec. 2: the M-cycle
 * repeated).  u holds the start state and receives the result; work is a second array of
 * the same shape whose ring already equals u's ring. */
void or_srj2d(int64_t nx, int64_t ny, double* u, const double* b, const double* wt, const double* c_seq,
              int64_t M, int64_t k0, int64_t nsweeps, double* work)
{
    double* cur = u;
    double* nxt = work;
    for (int64_t s = 0; s < nsweeps; ++s) {
        or_sweep2d(nx, ny, cur, b, wt, c_seq[(k0 + s) % M], nxt);
        double* t = cur; cur = nxt; nxt = t;
    }
    if (cur != u) memcpy(u, cur, sizeof(double) * (size_t)(nx + 2) * (size_t)(ny + 2));
}

void or_srj3d(int64_t nx, int64_t ny, int64_t nz, double* u, const double* b, const double* wt,
              const double* c_seq, int64_t M, int64_t k0, int64_t nsweeps, double* work)
{
    double* cur = u;
    double* nxt = work;
    for (int64_t s = 0; s < nsweeps; ++s) {
        or_sweep3d(nx, ny, nz, cur, b, wt, c_seq[(k0 + s) % M], nxt);
        double* t = cur; cur = nxt; nxt = t;
    }
    if (cur != u)
        memcpy(u, cur, sizeof(double) * (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(nz + 2));
}

/* ------------------------------------------------------------ residual norms */

/* Compensated (Kahan) accumulation, row by row, then over rows in order. */
typedef struct { double s, c; } kahan_t;
static inline void kadd(kahan_t* k, double x)
{
    double y = x - k->c;
    double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

/* r = b - A u = (s + b) - dg u on the interior.  out[0] = sum r^2, out[1] = max |r|. */
void or_residual2d(int64_t nx, int64_t ny, const double* u, const double* b, const double* wt, double* out,
                   double* rowsum, double* rowmax)
{
    const double wy = wt[0], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= ny; ++i) {
        kahan_t acc = {0.0, 0.0};
        double m = 0.0;
        for (int64_t j = 1; j <= nx; ++j) {
            double s = (u[I2(i, j - 1)] + u[I2(i, j + 1)]) + wy * (u[I2(i - 1, j)] + u[I2(i + 1, j)]);
            double r = (s + b[I2(i, j)]) - dg * u[I2(i, j)];
            kadd(&acc, r * r);
            double a = fabs(r);
            if (a > m || a != a) m = a;
        }
        rowsum[i - 1] = acc.s;
        rowmax[i - 1] = m;
    }
    kahan_t tot = {0.0, 0.0};
    double m = 0.0;
    for (int64_t i = 0; i < ny; ++i) {
        kadd(&tot, rowsum[i]);
        if (rowmax[i] > m || rowmax[i] != rowmax[i]) m = rowmax[i];
    }
    out[0] = tot.s;
    out[1] = m;
}

void or_residual3d(int64_t nx, int64_t ny, int64_t nz, const double* u, const double* b, const double* wt,
                   double* out, double* rowsum, double* rowmax)
{
    const double wy = wt[0], wz = wt[1], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k <= nz; ++k) {
        for (int64_t i = 1; i <= ny; ++i) {
            kahan_t acc = {0.0, 0.0};
            double m = 0.0;
            for (int64_t j = 1; j <= nx; ++j) {
                double s = ((u[I3(k, i, j - 1)] + u[I3(k, i, j + 1)]) +
                            wy * (u[I3(k, i - 1, j)] + u[I3(k, i + 1, j)])) +
                           wz * (u[I3(k - 1, i, j)] + u[I3(k + 1, i, j)]);
                double r = (s + b[I3(k, i, j)]) - dg * u[I3(k, i, j)];
                kadd(&acc, r * r);
                double a = fabs(r);
                if (a > m || a != a) m = a;
            }
            rowsum[(k - 1) * ny + (i - 1)] = acc.s;
            rowmax[(k - 1) * ny + (i - 1)] = m;
        }
    }
    kahan_t tot = {0.0, 0.0};
    double m = 0.0;
    for (int64_t i = 0; i < ny * nz; ++i) {
        kadd(&tot, rowsum[i]);
        if (rowmax[i] > m || rowmax[i] != rowmax[i]) m = rowmax[i];
    }
    out[0] = tot.s;
    out[1] = m;
}

/* r written out (interior; ring set to 0). */
void or_residual_field2d(int64_t nx, int64_t ny, const double* u, const double* b, const double* wt, double* r)
{
    const double wy = wt[0], dg = wt[2];
    memset(r, 0, sizeof(double) * (size_t)(nx + 2) * (size_t)(ny + 2));
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= ny; ++i)
        for (int64_t j = 1; j <= nx; ++j) {
            double s = (u[I2(i, j - 1)] + u[I2(i, j + 1)]) + wy * (u[I2(i - 1, j)] + u[I2(i + 1, j)]);
            r[I2(i, j)] = (s + b[I2(i, j)]) - dg * u[I2(i, j)];
        }
}

void or_residual_field3d(int64_t nx, int64_t ny, int64_t nz, const double* u, const double* b,
                         const double* wt, double* r)
{
    const double wy = wt[0], wz = wt[1], dg = wt[2];
    memset(r, 0, sizeof(double) * (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(nz + 2));
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k <= nz; ++k)
        for (int64_t i = 1; i <= ny; ++i)
            for (int64_t j = 1; j <= nx; ++j) {
                double s = ((u[I3(k, i, j - 1)] + u[I3(k, i, j + 1)]) +
                            wy * (u[I3(k, i - 1, j)] + u[I3(k, i + 1, j)])) +
                           wz * (u[I3(k - 1, i, j)] + u[I3(k + 1, i, j)]);
                r[I3(k, i, j)] = (s + b[I3(k, i, j)]) - dg * u[I3(k, i, j)];
            }
}

/* ------------------------------------------------- reduced-precision sweeps */
/* Same association, evaluated in binary32.  c and the weights wt = {wy, wz, dg} are the
 * binary32 roundings of their binary64 values. */

void or_sweep2d_f32(int64_t nx, int64_t ny, const float* u, const float* b, const float* wt, float c,
                    float* out)
{
    const float wy = wt[0], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= ny; ++i)
        for (int64_t j = 1; j <= nx; ++j) {
            float s = (u[I2(i, j - 1)] + u[I2(i, j + 1)]) + wy * (u[I2(i - 1, j)] + u[I2(i + 1, j)]);
            float t = (s + b[I2(i, j)]) - dg * u[I2(i, j)];
            out[I2(i, j)] = u[I2(i, j)] + c * t;
        }
}

void or_sweep3d_f32(int64_t nx, int64_t ny, int64_t nz, const float* u, const float* b, const float* wt,
                    float c, float* out)
{
    const float wy = wt[0], wz = wt[1], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k <= nz; ++k)
        for (int64_t i = 1; i <= ny; ++i)
            for (int64_t j = 1; j <= nx; ++j) {
                float s = ((u[I3(k, i, j - 1)] + u[I3(k, i, j + 1)]) +
                           wy * (u[I3(k, i - 1, j)] + u[I3(k, i + 1, j)])) +
                          wz * (u[I3(k - 1, i, j)] + u[I3(k + 1, i, j)]);
                float t = (s + b[I3(k, i, j)]) - dg * u[I3(k, i, j)];
                out[I3(k, i, j)] = u[I3(k, i, j)] + c * t;
            }
}

/* bfloat16 storage: the upper 16 bits of a binary32; widening is exact, narrowing rounds
 * to nearest, ties to even (quiet NaN kept quiet). */
static inline float bf_load(uint16_t h)
{
    uint32_t x = (uint32_t)h << 16;
    float f;
    memcpy(&f, &x, 4);
    return f;
}
static inline uint16_t bf_store(float f)
{
    uint32_t x;
    memcpy(&x, &f, 4);
    if ((x & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((x >> 16) | 0x40u);
    x += 0x7fffu + ((x >> 16) & 1u);
    return (uint16_t)(x >> 16);
}

void or_f32_to_bf16(int64_t n, const float* in, uint16_t* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bf_store(in[i]);
}
void or_bf16_to_f32(int64_t n, const uint16_t* in, float* out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = bf_load(in[i]);
}

void or_sweep2d_bf16(int64_t nx, int64_t ny, const uint16_t* u, const uint16_t* b, const float* wt, float c,
                     uint16_t* out)
{
    const float wy = wt[0], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= ny; ++i)
        for (int64_t j = 1; j <= nx; ++j) {
            float s = (bf_load(u[I2(i, j - 1)]) + bf_load(u[I2(i, j + 1)])) +
                      wy * (bf_load(u[I2(i - 1, j)]) + bf_load(u[I2(i + 1, j)]));
            float uc = bf_load(u[I2(i, j)]);
            float t = (s + bf_load(b[I2(i, j)])) - dg * uc;
            out[I2(i, j)] = bf_store(uc + c * t);
        }
}

void or_sweep3d_bf16(int64_t nx, int64_t ny, int64_t nz, const uint16_t* u, const uint16_t* b,
                     const float* wt, float c, uint16_t* out)
{
    const float wy = wt[0], wz = wt[1], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k <= nz; ++k)
        for (int64_t i = 1; i <= ny; ++i)
            for (int64_t j = 1; j <= nx; ++j) {
                float s = ((bf_load(u[I3(k, i, j - 1)]) + bf_load(u[I3(k, i, j + 1)])) +
                           wy * (bf_load(u[I3(k, i - 1, j)]) + bf_load(u[I3(k, i + 1, j)]))) +
                          wz * (bf_load(u[I3(k - 1, i, j)]) + bf_load(u[I3(k + 1, i, j)]));
                float uc = bf_load(u[I3(k, i, j)]);
                float t = (s + bf_load(b[I3(k, i, j)])) - dg * uc;
                out[I3(k, i, j)] = bf_store(uc + c * t);
            }
}

/* ------------------------------------------- homogeneous Neumann (Sec. 3.1 model problem) */
/* Cell-centred grid of n_i cells per axis; the ring holds ghost cells that mirror the
 * adjacent cell (zero normal derivative), so a neighbour across the boundary is the cell
 * itself.  The ring is never read.  Weights and association as the Dirichlet step. */

static inline double nb2(const double* u, int64_t nx, int64_t ny, int64_t i, int64_t j, int64_t di, int64_t dj)
{
    int64_t ii = i + di, jj = j + dj;
    if (ii < 1 || ii > ny) ii = i;
    if (jj < 1 || jj > nx) jj = j;
    return u[I2(ii, jj)];
}

static inline double nb3(const double* u, int64_t nx, int64_t ny, int64_t nz, int64_t k, int64_t i, int64_t j,
                         int64_t dk, int64_t di, int64_t dj)
{
    int64_t kk = k + dk, ii = i + di, jj = j + dj;
    if (kk < 1 || kk > nz) kk = k;
    if (ii < 1 || ii > ny) ii = i;
    if (jj < 1 || jj > nx) jj = j;
    return u[I3(kk, ii, jj)];
}

void or_sweep2d_neu(int64_t nx, int64_t ny, const double* u, const double* b, const double* wt, double c,
                    double* out)
{
    const double wy = wt[0], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t i = 1; i <= ny; ++i)
        for (int64_t j = 1; j <= nx; ++j) {
            double s = (nb2(u, nx, ny, i, j, 0, -1) + nb2(u, nx, ny, i, j, 0, 1)) +
                       wy * (nb2(u, nx, ny, i, j, -1, 0) + nb2(u, nx, ny, i, j, 1, 0));
            double t = (s + b[I2(i, j)]) - dg * u[I2(i, j)];
            out[I2(i, j)] = u[I2(i, j)] + c * t;
        }
}

void or_sweep3d_neu(int64_t nx, int64_t ny, int64_t nz, const double* u, const double* b, const double* wt,
                    double c, double* out)
{
    const double wy = wt[0], wz = wt[1], dg = wt[2];
#pragma omp parallel for schedule(static)
    for (int64_t k = 1; k <= nz; ++k)
        for (int64_t i = 1; i <= ny; ++i)
            for (int64_t j = 1; j <= nx; ++j) {
                double s = ((nb3(u, nx, ny, nz, k, i, j, 0, 0, -1) + nb3(u, nx, ny, nz, k, i, j, 0, 0, 1)) +
                            wy * (nb3(u, nx, ny, nz, k, i, j, 0, -1, 0) + nb3(u, nx, ny, nz, k, i, j, 0, 1, 0))) +
                           wz * (nb3(u, nx, ny, nz, k, i, j, -1, 0, 0) + nb3(u, nx, ny, nz, k, i, j, 1, 0, 0));
                double t = (s + b[I3(k, i, j)]) - dg * u[I3(k, i, j)];
                out[I3(k, i, j)] = u[I3(k, i, j)] + c * t;
            }
}

/* r = b - A u with the mirrored neighbours; field (ring 0) and, in out, sum r^2 (compensated
 * per line, then over lines) and max |r|. */
void or_residual_neu(int64_t nx, int64_t ny, int64_t nz, int ndim, const double* u, const double* b,
                     const double* wt, double* r, double* out, double* rowsum, double* rowmax)
{
    const double wy = wt[0], wz = wt[1], dg = wt[2];
    const int64_t planes = ndim == 3 ? nz : 1;
    memset(r, 0, sizeof(double) * (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(ndim == 3 ? nz + 2 : 1));
#pragma omp parallel for schedule(static)
    for (int64_t line = 0; line < planes * ny; ++line) {
        const int64_t k = ndim == 3 ? line / ny + 1 : 0, i = line % ny + 1;
        kahan_t acc = {0.0, 0.0};
        double m = 0.0;
        for (int64_t j = 1; j <= nx; ++j) {
            double s, uc, rv;
            size_t p;
            if (ndim == 3) {
                s = ((nb3(u, nx, ny, nz, k, i, j, 0, 0, -1) + nb3(u, nx, ny, nz, k, i, j, 0, 0, 1)) +
                     wy * (nb3(u, nx, ny, nz, k, i, j, 0, -1, 0) + nb3(u, nx, ny, nz, k, i, j, 0, 1, 0))) +
                    wz * (nb3(u, nx, ny, nz, k, i, j, -1, 0, 0) + nb3(u, nx, ny, nz, k, i, j, 1, 0, 0));
                p = I3(k, i, j);
            } else {
                s = (nb2(u, nx, ny, i, j, 0, -1) + nb2(u, nx, ny, i, j, 0, 1)) +
                    wy * (nb2(u, nx, ny, i, j, -1, 0) + nb2(u, nx, ny, i, j, 1, 0));
                p = I2(i, j);
            }
            uc = u[p];
            rv = (s + b[p]) - dg * uc;
            r[p] = rv;
            kadd(&acc, rv * rv);
            double a = fabs(rv);
            if (a > m || a != a) m = a;
        }
        rowsum[line] = acc.s;
        rowmax[line] = m;
    }
    kahan_t tot = {0.0, 0.0};
    double m = 0.0;
    for (int64_t line = 0; line < planes * ny; ++line) {
        kadd(&tot, rowsum[line]);
        if (rowmax[line] > m || rowmax[line] != rowmax[line]) m = rowmax[line];
    }
    out[0] = tot.s;
    out[1] = m;
}

/* ------------------------------------- variable-coefficient operators with a mask (Sec. 5.3) */
/* The operator (A u)_P = a_P u_P - sum_nb a_nb u_nb, given per point.  Jacobi-scaled: every
 * neighbour weight is w_nb = a_nb / a_P and the source is bs = f / a_P (one IEEE division
 * each), so one step with weight omega is
 *     s = (w_W W + w_E E) + (w_S S + w_N N)   [ + (w_D D + w_U U) in 3D ]
 *     t = (s + bs) - u ;   u' = u + omega * t
 * at every interior point whose mask is 0; masked points (mask != 0) and the ring keep their
 * values (Dirichlet data on an arbitrarily shaped boundary).  wts holds the 2d neighbour
 * weight arrays one after the other (W, E, S, N[, D, U]), each of the full-grid size. */

void or_op_scale(int64_t n, int nnb, const double* coef, double* wts, const double* f, double* bs)
{
    /* coef: a_P then the nnb neighbour arrays; f may be NULL */
    for (int64_t i = 0; i < n; ++i) {
        const double ap = coef[i];
        for (int k = 0; k < nnb; ++k) wts[(size_t)k * (size_t)n + (size_t)i] = coef[(size_t)(k + 1) * (size_t)n + (size_t)i] / ap;
        if (f) bs[i] = f[i] / ap;
    }
}

static inline double op_t(int ndim, int64_t nx, int64_t ny, int64_t nz, size_t p, const double* u, const double* wts,
                          const double* bs)
{
    const size_t n = (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(ndim == 3 ? nz + 2 : 1);
    const size_t px = (size_t)(nx + 2), pl = px * (size_t)(ny + 2);
    double s = (wts[p] * u[p - 1] + wts[n + p] * u[p + 1]) + (wts[2 * n + p] * u[p - px] + wts[3 * n + p] * u[p + px]);
    if (ndim == 3) s = s + (wts[4 * n + p] * u[p - pl] + wts[5 * n + p] * u[p + pl]);
    return (s + bs[p]) - u[p];
}

void or_op_sweep(int64_t nx, int64_t ny, int64_t nz, int ndim, const double* u, const double* wts, const double* bs,
                 const uint8_t* mask, double omega, double* out)
{
    const int64_t planes = ndim == 3 ? nz : 1;
#pragma omp parallel for schedule(static)
    for (int64_t line = 0; line < planes * ny; ++line) {
        const int64_t k = ndim == 3 ? line / ny + 1 : 0, i = line % ny + 1;
        for (int64_t j = 1; j <= nx; ++j) {
            const size_t p = ndim == 3 ? I3(k, i, j) : I2(i, j);
            if (mask && mask[p]) {
                out[p] = u[p];
                continue;
            }
            out[p] = u[p] + omega * op_t(ndim, nx, ny, nz, p, u, wts, bs);
        }
    }
}

/* Jacobi-scaled residual t (0 at masked points and on the ring) into r (may be NULL), with
 * out[0] = sum t^2 (compensated per line) and out[1] = max |t|.  zero_free: read u as 0 at the
 * interior points the sweep updates (giving the scaled source plus boundary terms). */
void or_op_residual(int64_t nx, int64_t ny, int64_t nz, int ndim, const double* u, const double* wts,
                    const double* bs, const uint8_t* mask, int zero_free, double* r, double* out, double* rowsum,
                    double* rowmax, double* scratch)
{
    const int64_t planes = ndim == 3 ? nz : 1;
    const size_t n = (size_t)(nx + 2) * (size_t)(ny + 2) * (size_t)(ndim == 3 ? nz + 2 : 1);
    const double* v = u;
    if (zero_free) {
        memcpy(scratch, u, sizeof(double) * n);
        for (int64_t line = 0; line < planes * ny; ++line) {
            const int64_t k = ndim == 3 ? line / ny + 1 : 0, i = line % ny + 1;
            for (int64_t j = 1; j <= nx; ++j) {
                const size_t p = ndim == 3 ? I3(k, i, j) : I2(i, j);
                if (!(mask && mask[p])) scratch[p] = 0.0;
            }
        }
        v = scratch;
    }
    if (r) memset(r, 0, sizeof(double) * n);
#pragma omp parallel for schedule(static)
    for (int64_t line = 0; line < planes * ny; ++line) {
        const int64_t k = ndim == 3 ? line / ny + 1 : 0, i = line % ny + 1;
        kahan_t acc = {0.0, 0.0};
        double m = 0.0;
        for (int64_t j = 1; j <= nx; ++j) {
            const size_t p = ndim == 3 ? I3(k, i, j) : I2(i, j);
            const double t = (mask && mask[p]) ? 0.0 : op_t(ndim, nx, ny, nz, p, v, wts, bs);
            if (r) r[p] = t;
            kadd(&acc, t * t);
            const double a = fabs(t);
            if (a > m || a != a) m = a;
        }
        rowsum[line] = acc.s;
        rowmax[line] = m;
    }
    kahan_t tot = {0.0, 0.0};
    double m = 0.0;
    for (int64_t line = 0; line < planes * ny; ++line) {
        kadd(&tot, rowsum[line]);
        if (rowmax[line] > m || rowmax[line] != rowmax[line]) m = rowmax[line];
    }
    out[0] = tot.s;
    out[1] = m;
}
