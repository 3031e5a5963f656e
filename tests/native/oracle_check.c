/* Host-side check of the oracle's C loops, built with address and undefined-behaviour
 * sanitizers by tests/test_sanitizers.py.  Runs every sweep, residual and conversion routine
 * on small grids whose arrays are allocated to their exact sizes (so a read or write one
 * element outside a grid is reported), in the smallest shapes too (n = 1), and checks a
 * weight-1 step against the Jacobi step. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_sweep2d(int64_t, int64_t, const double*, const double*, const double*, double, double*);
void or_sweep3d(int64_t, int64_t, int64_t, const double*, const double*, const double*, double, double*);
void or_jacobi2d(int64_t, int64_t, const double*, const double*, double*);
void or_jacobi3d(int64_t, int64_t, int64_t, const double*, const double*, double*);
void or_srj2d(int64_t, int64_t, double*, const double*, const double*, const double*, int64_t, int64_t, int64_t,
              double*);
void or_srj3d(int64_t, int64_t, int64_t, double*, const double*, const double*, const double*, int64_t, int64_t,
              int64_t, double*);
void or_residual2d(int64_t, int64_t, const double*, const double*, const double*, double*, double*, double*);
void or_residual3d(int64_t, int64_t, int64_t, const double*, const double*, const double*, double*, double*,
                   double*);
void or_residual_field2d(int64_t, int64_t, const double*, const double*, const double*, double*);
void or_residual_field3d(int64_t, int64_t, int64_t, const double*, const double*, const double*, double*);
void or_sweep2d_f32(int64_t, int64_t, const float*, const float*, const float*, float, float*);
void or_sweep3d_f32(int64_t, int64_t, int64_t, const float*, const float*, const float*, float, float*);
void or_sweep2d_bf16(int64_t, int64_t, const uint16_t*, const uint16_t*, const float*, float, uint16_t*);
void or_sweep3d_bf16(int64_t, int64_t, int64_t, const uint16_t*, const uint16_t*, const float*, float, uint16_t*);
void or_f32_to_bf16(int64_t, const float*, uint16_t*);
void or_bf16_to_f32(int64_t, const uint16_t*, float*);

static double* filled(size_t n, unsigned* seed)
{
    double* a = (double*)malloc(n * sizeof(double));
    for (size_t i = 0; i < n; ++i) {
        *seed = *seed * 1103515245u + 12345u;
        a[i] = ((*seed >> 8) & 0xffff) / 32768.0 - 1.0;
    }
    return a;
}

int main(void)
{
    int bad = 0;
    unsigned seed = 7;
    const int64_t shapes[][3] = {{1, 1, 1}, {3, 2, 4}, {17, 9, 5}};
    for (int s = 0; s < 3; ++s) {
        const int64_t nx = shapes[s][0], ny = shapes[s][1], nz = shapes[s][2];
        const size_t n2 = (size_t)(nx + 2) * (size_t)(ny + 2), n3 = n2 * (size_t)(nz + 2);
        double *u = filled(n3, &seed), *b = filled(n3, &seed), *o = filled(n3, &seed), *j = filled(n3, &seed);
        double *w = filled(n3, &seed), *rs = filled((size_t)(ny * nz), &seed), *rm = filled((size_t)(ny * nz), &seed);
        double out[2], c[3] = {0.25, 2.5, 0.1};
        const double w2[3] = {1.0, 1.0, 4.0}, w3[3] = {1.0, 1.0, 6.0}, wa[3] = {0.25, 3.0, 8.5};
        const float f2[3] = {1.0f, 1.0f, 4.0f}, f3[3] = {0.25f, 3.0f, 8.5f};
        or_sweep2d(nx, ny, u, b, w2, 0.25, o);
        or_jacobi2d(nx, ny, u, b, j);
        for (int64_t i = 1; i <= ny; ++i)
            for (int64_t k = 1; k <= nx; ++k) {
                const size_t p = (size_t)i * (size_t)(nx + 2) + (size_t)k;
                if (fabs(o[p] - j[p]) > 1e-15 * (1.0 + fabs(j[p]))) ++bad;
            }
        or_sweep3d(nx, ny, nz, u, b, w3, 1.0 / 6.0, o);
        or_sweep3d(nx, ny, nz, u, b, wa, 0.3, o);
        or_jacobi3d(nx, ny, nz, u, b, j);
        or_residual2d(nx, ny, u, b, wa, out, rs, rm);
        or_residual3d(nx, ny, nz, u, b, wa, out, rs, rm);
        or_residual_field2d(nx, ny, u, b, wa, o);
        or_residual_field3d(nx, ny, nz, u, b, wa, o);
        for (size_t i = 0; i < n3; ++i) w[i] = u[i];
        or_srj2d(nx, ny, u, b, wa, c, 3, 1, 5, w);
        for (size_t i = 0; i < n3; ++i) w[i] = u[i];
        or_srj3d(nx, ny, nz, u, b, w3, c, 3, 2, 4, w);
        float *u32 = (float*)malloc(n3 * sizeof(float)), *b32 = (float*)malloc(n3 * sizeof(float));
        float* o32 = (float*)malloc(n3 * sizeof(float));
        uint16_t *ub = (uint16_t*)malloc(n3 * 2), *bb = (uint16_t*)malloc(n3 * 2), *ob = (uint16_t*)malloc(n3 * 2);
        for (size_t i = 0; i < n3; ++i) {
            u32[i] = (float)u[i];
            b32[i] = (float)b[i];
        }
        or_sweep2d_f32(nx, ny, u32, b32, f2, 3.0f, o32);
        or_sweep3d_f32(nx, ny, nz, u32, b32, f3, 3.0f, o32);
        or_f32_to_bf16((int64_t)n3, u32, ub);
        or_f32_to_bf16((int64_t)n3, b32, bb);
        or_sweep2d_bf16(nx, ny, ub, bb, f3, 3.0f, ob);
        or_sweep3d_bf16(nx, ny, nz, ub, bb, f2, 3.0f, ob);
        or_bf16_to_f32((int64_t)n3, ob, o32);
        free(u32); free(b32); free(o32); free(ub); free(bb); free(ob);
        free(u); free(b); free(o); free(j); free(w); free(rs); free(rm);
        (void)n2;
    }
    printf("%s\n", bad ? "FAILED" : "ok");
    return bad ? 1 : 0;
}
