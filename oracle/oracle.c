/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the iterated
 * 3D 7-point smoothers (Treibig, Wellein, Hager: "Efficient multicore-aware
 * parallelization strategies for iterative stencil computations").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library (paper_1004_1741_amd/) and must never be used as a fallback
 * for it.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (OpenMP is used only by oracle_jacobi_f64_threads, the CPU baseline)
 * (no FMA contraction, no reassociation, SSE2 doubles, round-to-nearest-even).
 *
 * Grid layout: interior extents nx, ny, nz and a ghost layer of width h >= 1;
 * a C array of (nz+2h)*(ny+2h)*(nx+2h) values, x contiguous:
 *     index(k, j, i) = (k*(ny+2h) + j)*(nx+2h) + i
 * with interior i in [h, h+nx), j in [h, h+ny), k in [h, h+nz).  Ghost cells
 * hold Dirichlet values and are never written.  A right-hand side f, when
 * given, is interior-only, nz*ny*nx values, x contiguous.
 *
 * Update of one site (Sec. 3, Jacobi and Gauss-Seidel loop nests; the
 * right-hand-side term is the Poisson form the paper names but does not print):
 *     s = ((((x- + x+) + y-) + y+) + z-) + z+
 *     v = (a*c) + (b*s)          [the a*c term is omitted when a == 0]
 *     v = v + (g*f)              [only when f is given]
 * The neighbour sum follows C left-to-right association of the printed
 * expressions.  Jacobi reads every operand from the previous sweep and writes
 * a second array; Gauss-Seidel updates in place in lexicographic order (i
 * fastest, then j, then k, all increasing), so x-, y-, z- are already new and
 * x+, y+, z+ are still old.
 *
 * Red-black Gauss-Seidel (the common alternative ordering the paper names
 * next to the lexicographic one) colours sites by the parity of i + j + k.
 *
 * parity pins: tests/test_oracle.py (closed-form Jacobi decay of discrete sine
 * modes, harmonic fixed points, exact rational arithmetic with dyadic weights,
 * brute-force loop transcriptions, split invariance, defect-correction
 * equivalence, Gauss-Seidel asymptotic rate).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IDX(k, j, i) ((((int64_t)(k)) * py + (j)) * px + (i))
#define FIDX(k, j, i) ((((int64_t)(k) - h) * ny + ((j) - h)) * nx + ((i) - h))

/* ---------------------------------------------------------------- FP64 ---- */

/* Jacobi, Sec. 3: `sweeps` out-of-place sweeps; result returned in u. */
int oracle_jacobi_f64(int64_t nx, int64_t ny, int64_t nz, int64_t h, double *u,
                      const double *f, double a, double b, double g, int sweeps)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h, pz = nz + 2 * h;
    const int64_t n = px * py * pz;
    double *src = u;
    double *dst = (double *)malloc((size_t)n * sizeof(double));
    if (!dst) return -2;
    memcpy(dst, u, (size_t)n * sizeof(double)); /* identical ghost cells */
    for (int it = 0; it < sweeps; it++) {
        for (int64_t k = h; k < h + nz; k++)
            for (int64_t j = h; j < h + ny; j++)
                for (int64_t i = h; i < h + nx; i++) {
                    double s = src[IDX(k, j, i - 1)];
                    s = s + src[IDX(k, j, i + 1)];
                    s = s + src[IDX(k, j - 1, i)];
                    s = s + src[IDX(k, j + 1, i)];
                    s = s + src[IDX(k - 1, j, i)];
                    s = s + src[IDX(k + 1, j, i)];
                    double v;
                    if (a != 0.0)
                        v = (a * src[IDX(k, j, i)]) + (b * s);
                    else
                        v = b * s;
                    if (f) v = v + (g * f[FIDX(k, j, i)]);
                    dst[IDX(k, j, i)] = v;
                }
        double *t = src; src = dst; dst = t;
    }
    if (src != u) {
        memcpy(u, src, (size_t)n * sizeof(double));
        free(src);
    } else {
        free(dst);
    }
    return 0;
}

/* CPU baseline: the Jacobi loop nest above without a right-hand side, its k
 * loop split across OpenMP threads.  Every site sees the same operations in
 * the same order, so the result equals oracle_jacobi_f64 for any thread
 * count.  nthreads <= 0 means the OpenMP default.  Returns the number of
 * threads used, or -2 if the second array cannot be allocated. */
int oracle_jacobi_f64_threads(int64_t nx, int64_t ny, int64_t nz, int64_t h, double *u,
                              double a, double b, int sweeps, int nthreads)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h, pz = nz + 2 * h;
    const int64_t n = px * py * pz;
    double *src = u;
    double *dst = (double *)malloc((size_t)n * sizeof(double));
    int used = 1;
    if (!dst) return -2;
    memcpy(dst, u, (size_t)n * sizeof(double));
    for (int it = 0; it < sweeps; it++) {
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
#endif
        for (int64_t k = h; k < h + nz; k++) {
#ifdef _OPENMP
            if (k == h) used = omp_get_num_threads();
#endif
            for (int64_t j = h; j < h + ny; j++)
                for (int64_t i = h; i < h + nx; i++) {
                    double s = src[IDX(k, j, i - 1)];
                    s = s + src[IDX(k, j, i + 1)];
                    s = s + src[IDX(k, j - 1, i)];
                    s = s + src[IDX(k, j + 1, i)];
                    s = s + src[IDX(k - 1, j, i)];
                    s = s + src[IDX(k + 1, j, i)];
                    dst[IDX(k, j, i)] = (a != 0.0) ? (a * src[IDX(k, j, i)]) + (b * s) : b * s;
                }
        }
        double *t = src; src = dst; dst = t;
    }
    if (src != u) {
        memcpy(u, src, (size_t)n * sizeof(double));
        free(src);
    } else {
        free(dst);
    }
    return used;
}

/* Lexicographic Gauss-Seidel, Sec. 3: `sweeps` in-place sweeps. */
int oracle_gs_f64(int64_t nx, int64_t ny, int64_t nz, int64_t h, double *u,
                  const double *f, double a, double b, double g, int sweeps)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    for (int it = 0; it < sweeps; it++) {
        for (int64_t k = h; k < h + nz; k++)
            for (int64_t j = h; j < h + ny; j++)
                for (int64_t i = h; i < h + nx; i++) {
                    double s = u[IDX(k, j, i - 1)];
                    s = s + u[IDX(k, j, i + 1)];
                    s = s + u[IDX(k, j - 1, i)];
                    s = s + u[IDX(k, j + 1, i)];
                    s = s + u[IDX(k - 1, j, i)];
                    s = s + u[IDX(k + 1, j, i)];
                    double v;
                    if (a != 0.0)
                        v = (a * u[IDX(k, j, i)]) + (b * s);
                    else
                        v = b * s;
                    if (f) v = v + (g * f[FIDX(k, j, i)]);
                    u[IDX(k, j, i)] = v;
                }
    }
    return 0;
}

/* Red-black Gauss-Seidel: one sweep updates, in place, first every "red"
 * site ((i + j + k) even, interior coordinates counted from 0) and then every
 * "black" site, each with the same update as above.  Axis neighbours always
 * have the other colour, so red sites read only old black values and black
 * sites read the new red ones; the loop order within a colour is free. */
int oracle_rbgs_f64(int64_t nx, int64_t ny, int64_t nz, int64_t h, double *u,
                    const double *f, double a, double b, double g, int sweeps)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    for (int it = 0; it < sweeps; it++)
        for (int color = 0; color < 2; color++)
            for (int64_t k = h; k < h + nz; k++)
                for (int64_t j = h; j < h + ny; j++)
                    for (int64_t i = h; i < h + nx; i++) {
                        if ((((i - h) + (j - h) + (k - h)) & 1) != color) continue;
                        double s = u[IDX(k, j, i - 1)];
                        s = s + u[IDX(k, j, i + 1)];
                        s = s + u[IDX(k, j - 1, i)];
                        s = s + u[IDX(k, j + 1, i)];
                        s = s + u[IDX(k - 1, j, i)];
                        s = s + u[IDX(k + 1, j, i)];
                        double v;
                        if (a != 0.0)
                            v = (a * u[IDX(k, j, i)]) + (b * s);
                        else
                            v = b * s;
                        if (f) v = v + (g * f[FIDX(k, j, i)]);
                        u[IDX(k, j, i)] = v;
                    }
    return 0;
}

/* ---------------------------------------------------------------- FP32 ---- */
/* Same loops with float storage and float arithmetic; weights are rounded to
 * float once (round-to-nearest-even). */

int oracle_jacobi_f32(int64_t nx, int64_t ny, int64_t nz, int64_t h, float *u,
                      const float *f, double a64, double b64, double g64, int sweeps)
{
    const float a = (float)a64, b = (float)b64, g = (float)g64;
    const int64_t px = nx + 2 * h, py = ny + 2 * h, pz = nz + 2 * h;
    const int64_t n = px * py * pz;
    float *src = u;
    float *dst = (float *)malloc((size_t)n * sizeof(float));
    if (!dst) return -2;
    memcpy(dst, u, (size_t)n * sizeof(float));
    for (int it = 0; it < sweeps; it++) {
        for (int64_t k = h; k < h + nz; k++)
            for (int64_t j = h; j < h + ny; j++)
                for (int64_t i = h; i < h + nx; i++) {
                    float s = src[IDX(k, j, i - 1)];
                    s = s + src[IDX(k, j, i + 1)];
                    s = s + src[IDX(k, j - 1, i)];
                    s = s + src[IDX(k, j + 1, i)];
                    s = s + src[IDX(k - 1, j, i)];
                    s = s + src[IDX(k + 1, j, i)];
                    float v;
                    if (a != 0.0f)
                        v = (a * src[IDX(k, j, i)]) + (b * s);
                    else
                        v = b * s;
                    if (f) v = v + (g * f[FIDX(k, j, i)]);
                    dst[IDX(k, j, i)] = v;
                }
        float *t = src; src = dst; dst = t;
    }
    if (src != u) {
        memcpy(u, src, (size_t)n * sizeof(float));
        free(src);
    } else {
        free(dst);
    }
    return 0;
}

int oracle_gs_f32(int64_t nx, int64_t ny, int64_t nz, int64_t h, float *u,
                  const float *f, double a64, double b64, double g64, int sweeps)
{
    const float a = (float)a64, b = (float)b64, g = (float)g64;
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    for (int it = 0; it < sweeps; it++) {
        for (int64_t k = h; k < h + nz; k++)
            for (int64_t j = h; j < h + ny; j++)
                for (int64_t i = h; i < h + nx; i++) {
                    float s = u[IDX(k, j, i - 1)];
                    s = s + u[IDX(k, j, i + 1)];
                    s = s + u[IDX(k, j - 1, i)];
                    s = s + u[IDX(k, j + 1, i)];
                    s = s + u[IDX(k - 1, j, i)];
                    s = s + u[IDX(k + 1, j, i)];
                    float v;
                    if (a != 0.0f)
                        v = (a * u[IDX(k, j, i)]) + (b * s);
                    else
                        v = b * s;
                    if (f) v = v + (g * f[FIDX(k, j, i)]);
                    u[IDX(k, j, i)] = v;
                }
    }
    return 0;
}

/* Red-black Gauss-Seidel in float (see oracle_rbgs_f64). */
int oracle_rbgs_f32(int64_t nx, int64_t ny, int64_t nz, int64_t h, float *u,
                    const float *f, double a64, double b64, double g64, int sweeps)
{
    const float a = (float)a64, b = (float)b64, g = (float)g64;
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    for (int it = 0; it < sweeps; it++)
        for (int color = 0; color < 2; color++)
            for (int64_t k = h; k < h + nz; k++)
                for (int64_t j = h; j < h + ny; j++)
                    for (int64_t i = h; i < h + nx; i++) {
                        if ((((i - h) + (j - h) + (k - h)) & 1) != color) continue;
                        float s = u[IDX(k, j, i - 1)];
                        s = s + u[IDX(k, j, i + 1)];
                        s = s + u[IDX(k, j - 1, i)];
                        s = s + u[IDX(k, j + 1, i)];
                        s = s + u[IDX(k - 1, j, i)];
                        s = s + u[IDX(k + 1, j, i)];
                        float v;
                        if (a != 0.0f)
                            v = (a * u[IDX(k, j, i)]) + (b * s);
                        else
                            v = b * s;
                        if (f) v = v + (g * f[FIDX(k, j, i)]);
                        u[IDX(k, j, i)] = v;
                    }
    return 0;
}

/* ----------------------------------------------------------- residuals ---- */

/* Sum of squares in index order (plain sequential FP64 accumulation). */
double oracle_sumsq(const double *x, int64_t n)
{
    double acc = 0.0;
    for (int64_t q = 0; q < n; q++) acc = acc + x[q] * x[q];
    return acc;
}

/* Residual of the h^2-scaled Poisson system A u = f' with A u = 6c - s:
 *     r = f' - ((6*c) - s),  s the neighbour sum in the order above.
 * f' is interior-only.  Writes r (interior-only) when r != NULL and returns
 * the lexicographic sum of r^2. */
double oracle_residual_f64(int64_t nx, int64_t ny, int64_t nz, int64_t h, const double *u,
                           const double *fp, double *r)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    double acc = 0.0;
    for (int64_t k = h; k < h + nz; k++)
        for (int64_t j = h; j < h + ny; j++)
            for (int64_t i = h; i < h + nx; i++) {
                double s = u[IDX(k, j, i - 1)];
                s = s + u[IDX(k, j, i + 1)];
                s = s + u[IDX(k, j - 1, i)];
                s = s + u[IDX(k, j + 1, i)];
                s = s + u[IDX(k - 1, j, i)];
                s = s + u[IDX(k + 1, j, i)];
                double c = u[IDX(k, j, i)];
                double fv = fp ? fp[FIDX(k, j, i)] : 0.0;
                double rv = fv - ((6.0 * c) - s);
                if (r) r[FIDX(k, j, i)] = rv;
                acc = acc + rv * rv;
            }
    return acc;
}

/* One-sweep defect of a general smoother u <- (a*c) + (b*s) [+ g*f]:
 *     r = (one update of u) - c      (interior-only output).
 * A further correction e from  e <- (a*e) + (b*s_e) + r,  e0 = 0, zero ghosts,
 * satisfies u0 + e_m = u_m for m sweeps in exact arithmetic. */
int oracle_defect_f64(int64_t nx, int64_t ny, int64_t nz, int64_t h, const double *u,
                      const double *f, double a, double b, double g, double *r)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    for (int64_t k = h; k < h + nz; k++)
        for (int64_t j = h; j < h + ny; j++)
            for (int64_t i = h; i < h + nx; i++) {
                double s = u[IDX(k, j, i - 1)];
                s = s + u[IDX(k, j, i + 1)];
                s = s + u[IDX(k, j - 1, i)];
                s = s + u[IDX(k, j + 1, i)];
                s = s + u[IDX(k - 1, j, i)];
                s = s + u[IDX(k + 1, j, i)];
                double c = u[IDX(k, j, i)];
                double v;
                if (a != 0.0)
                    v = (a * c) + (b * s);
                else
                    v = b * s;
                if (f) v = v + (g * f[FIDX(k, j, i)]);
                r[FIDX(k, j, i)] = v - c;
            }
    return 0;
}

/* -------------------------------------------------- iterative refinement ---- */

/* Defect-correction loop for the h^2-scaled Poisson system (method 0 =
 * Jacobi, 1 = lexicographic Gauss-Seidel, 2 = red-black Gauss-Seidel as the
 * inner smoother):
 *     loop: r = f' - A u; stop when ||r||/||f'|| <= tol;
 *           e = m sweeps of the smoother on A e = r from e = 0, zero ghosts,
 *               weights (a, b, g) = (0, 1/6, 1/6);
 *           u = u + e.
 * inner_f32 = 0: e, r and the sweeps in FP64 (the plain FP64 method);
 * inner_f32 = 1: r rounded to float, e and the sweeps in float, the
 *                correction added back in FP64.
 * Returns 0 on convergence, -6 when max_outer corrections were applied without
 * reaching tol.  *outer_done = corrections applied, *rel_out = last ||r||/||f'||. */
int oracle_refine(int64_t nx, int64_t ny, int64_t nz, int64_t h, int method, double *u,
                  const double *fp, int inner_f32, int m, double tol, int max_outer,
                  int *outer_done, double *rel_out)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h, pz = nz + 2 * h;
    const int64_t n = px * py * pz, ni = nx * ny * nz;
    double *r = (double *)malloc((size_t)ni * sizeof(double));
    double *e = (double *)malloc((size_t)n * sizeof(double));
    float *r32 = (float *)malloc((size_t)ni * sizeof(float));
    float *e32 = (float *)malloc((size_t)n * sizeof(float));
    if (!r || !e || !r32 || !e32) { free(r); free(e); free(r32); free(e32); return -2; }
    const double nf = sqrt(oracle_sumsq(fp, ni));
    int status = -6, outer = 0;
    double rel = INFINITY;
    for (;;) {
        double rr = oracle_residual_f64(nx, ny, nz, h, u, fp, r);
        rel = sqrt(rr) / nf;
        if (rel <= tol) { status = 0; break; }
        if (outer >= max_outer) break;
        if (inner_f32) {
            for (int64_t q = 0; q < ni; q++) r32[q] = (float)r[q];
            memset(e32, 0, (size_t)n * sizeof(float));
            if (method == 0)
                oracle_jacobi_f32(nx, ny, nz, h, e32, r32, 0.0, 1.0 / 6.0, 1.0 / 6.0, m);
            else if (method == 2)
                oracle_rbgs_f32(nx, ny, nz, h, e32, r32, 0.0, 1.0 / 6.0, 1.0 / 6.0, m);
            else
                oracle_gs_f32(nx, ny, nz, h, e32, r32, 0.0, 1.0 / 6.0, 1.0 / 6.0, m);
            for (int64_t k = h; k < h + nz; k++)
                for (int64_t j = h; j < h + ny; j++)
                    for (int64_t i = h; i < h + nx; i++)
                        u[IDX(k, j, i)] = u[IDX(k, j, i)] + (double)e32[IDX(k, j, i)];
        } else {
            memset(e, 0, (size_t)n * sizeof(double));
            if (method == 0)
                oracle_jacobi_f64(nx, ny, nz, h, e, r, 0.0, 1.0 / 6.0, 1.0 / 6.0, m);
            else if (method == 2)
                oracle_rbgs_f64(nx, ny, nz, h, e, r, 0.0, 1.0 / 6.0, 1.0 / 6.0, m);
            else
                oracle_gs_f64(nx, ny, nz, h, e, r, 0.0, 1.0 / 6.0, 1.0 / 6.0, m);
            for (int64_t k = h; k < h + nz; k++)
                for (int64_t j = h; j < h + ny; j++)
                    for (int64_t i = h; i < h + nx; i++)
                        u[IDX(k, j, i)] = u[IDX(k, j, i)] + e[IDX(k, j, i)];
        }
        outer++;
    }
    free(r); free(e); free(r32); free(e32);
    if (outer_done) *outer_done = outer;
    if (rel_out) *rel_out = rel;
    return status;
}

/* A smoothing job run in FP32-refined precision: one defect-correction step.
 *     r  = (one FP64 update of u0) - u0          (oracle_defect_f64)
 *     e  = `sweeps` float sweeps of the method on e <- (a*e) + (b*s_e) + (1*r32),
 *          e0 = 0, zero ghosts, r32 = float(r)
 *     u  = u0 + double(e)
 * Equal to `sweeps` plain sweeps from u0 in exact arithmetic. */
int oracle_refined_job(int64_t nx, int64_t ny, int64_t nz, int64_t h, int method, double *u,
                       const double *f, double a, double b, double g, int sweeps)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h, pz = nz + 2 * h;
    const int64_t n = px * py * pz, ni = nx * ny * nz;
    double *r = (double *)malloc((size_t)ni * sizeof(double));
    float *r32 = (float *)malloc((size_t)ni * sizeof(float));
    float *e32 = (float *)calloc((size_t)n, sizeof(float));
    if (!r || !r32 || !e32) { free(r); free(r32); free(e32); return -2; }
    oracle_defect_f64(nx, ny, nz, h, u, f, a, b, g, r);
    for (int64_t q = 0; q < ni; q++) r32[q] = (float)r[q];
    if (method == 0)
        oracle_jacobi_f32(nx, ny, nz, h, e32, r32, a, b, 1.0, sweeps);
    else if (method == 2)
        oracle_rbgs_f32(nx, ny, nz, h, e32, r32, a, b, 1.0, sweeps);
    else
        oracle_gs_f32(nx, ny, nz, h, e32, r32, a, b, 1.0, sweeps);
    for (int64_t k = h; k < h + nz; k++)
        for (int64_t j = h; j < h + ny; j++)
            for (int64_t i = h; i < h + nx; i++)
                u[IDX(k, j, i)] = u[IDX(k, j, i)] + (double)e32[IDX(k, j, i)];
    free(r); free(r32); free(e32);
    return 0;
}
