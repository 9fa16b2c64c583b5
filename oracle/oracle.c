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


/* ------------------------------------------------------------ multigrid ---- */
/*
 * Geometric multigrid V-cycle for the h^2-scaled Poisson system A u = f'
 * (A u = 6c - s), the solver the smoothers of Sec. 3 are built for (Sec. 1
 * names multigrid as their main user).  Textbook components, written out:
 *
 *   levels:  interior points n on (0, 1) at x_i = i/(n+1), i = 1..n, Dirichlet
 *            zero at i = 0 and n+1.  The next level has nc = floor((n+1)/2) - 1
 *            points per axis (coarsening while every axis has >= 3); when n+1
 *            is even the coarse points are the even fine points (nested), else
 *            (e.g. n = 512) the coarse spacing 1/(nc+1) is slightly more than
 *            twice the fine one and the transfers below interpolate
 *            geometrically.
 *   transfer weights (per axis): fine point i lies on the coarse grid at
 *            i (nc+1)/(n+1) = I0 + q/(n+1) with q = i (nc+1) mod (n+1); its
 *            linear interpolation weights are wm = (n+1-q)/(n+1) on coarse I0
 *            and wq = q/(n+1) on I0+1 (each one rounded division in the
 *            level's precision; coarse ghosts I = 0 and nc+1 are 0).
 *   prolongation P: trilinear interpolation, along x, then y, then z, each
 *            step (wm * lo) + (wq * hi); the result is added to the fine
 *            correction.
 *   restriction:  the transpose of P times `scale`, scale = (h/H) for the
 *            h^2-scaled coarse system (= rho = (nc+1)/(n+1) when the three axes
 *            share it, else the cube root of their product, computed in FP64
 *            and rounded once to the level precision).  Evaluated as x-sums
 *            over the fine points with a non-zero weight (increasing i,
 *            acc = acc + (w * r) from 0), then y-sums of those, then z, then
 *            times scale.  Nested levels give full weighting, 4 * (1/64)
 *            [1 2 1] x [1 2 1] x [1 2 1].
 *   smoother: 0 = weighted Jacobi with omega = 6/7 (a = b = g = 1/7),
 *            1 = lexicographic Gauss-Seidel, 2 = red-black Gauss-Seidel
 *            (a = 0, b = g = 1/6); the level's right-hand side is f.
 *   residual: res = r - ((6*c) - s) in the level's precision.
 * V-cycle at level l with right-hand side r_l:  e_l = 0; `pre` sweeps;
 * r_{l+1} = restricted residual; V-cycle at l+1; e_l += P e_{l+1}; `post`
 * sweeps.  The coarsest level runs `coarse` sweeps from e = 0.  Outer loop:
 * the defect correction of oracle_refine with one V-cycle as the inner solve
 * (inner_f32 = 1: r rounded to float, the whole V-cycle in float; 0: FP64).
 */

int64_t oracle_mg_coarse_n(int64_t n) { return (n + 1) / 2 - 1; }

/* coarse position of fine point i: I0 and q */
static void mg_pos(int64_t i, int64_t n, int64_t nc, int64_t *I0, int64_t *q)
{
    *I0 = (i * (nc + 1)) / (n + 1);
    *q = (i * (nc + 1)) % (n + 1);
}

/* fine points i with a non-zero weight towards coarse point I: [lo, hi] */
static void mg_support(int64_t I, int64_t n, int64_t nc, int64_t *lo, int64_t *hi)
{
    *lo = ((I - 1) * (n + 1)) / (nc + 1) + 1;
    *hi = ((I + 1) * (n + 1) - 1) / (nc + 1);
    if (*lo < 1) *lo = 1;
    if (*hi > n) *hi = n;
}

static double mg_w64(int64_t i, int64_t I, int64_t n, int64_t nc)
{
    int64_t I0, q;
    mg_pos(i, n, nc, &I0, &q);
    if (I == I0) return (double)(n + 1 - q) / (double)(n + 1);
    if (I == I0 + 1) return (double)q / (double)(n + 1);
    return 0.0;
}

static float mg_w32(int64_t i, int64_t I, int64_t n, int64_t nc)
{
    int64_t I0, q;
    mg_pos(i, n, nc, &I0, &q);
    if (I == I0) return (float)(n + 1 - q) / (float)(n + 1);
    if (I == I0 + 1) return (float)q / (float)(n + 1);
    return 0.0f;
}

/* h/H scale of the restriction between a fine level and the next one */
double oracle_mg_scale(int64_t nx, int64_t ny, int64_t nz)
{
    const double rx = (double)(oracle_mg_coarse_n(nx) + 1) / (double)(nx + 1);
    const double ry = (double)(oracle_mg_coarse_n(ny) + 1) / (double)(ny + 1);
    const double rz = (double)(oracle_mg_coarse_n(nz) + 1) / (double)(nz + 1);
    if (rx == ry && ry == rz) return rx;
    return cbrt(rx * ry * rz);
}

#define MG_FI(i, j, k) ((((k) - 1) * fny + ((j) - 1)) * fnx + ((i) - 1))

/* rc = scale * P^T res; res and rc interior-only. */
void oracle_mg_restrict_f64(int64_t fnx, int64_t fny, int64_t fnz, const double *res, double *rc,
                            double scale)
{
    const int64_t cnx = oracle_mg_coarse_n(fnx), cny = oracle_mg_coarse_n(fny),
                  cnz = oracle_mg_coarse_n(fnz);
    for (int64_t K = 1; K <= cnz; K++)
        for (int64_t J = 1; J <= cny; J++)
            for (int64_t I = 1; I <= cnx; I++) {
                int64_t i0, i1, j0, j1, k0, k1;
                mg_support(I, fnx, cnx, &i0, &i1);
                mg_support(J, fny, cny, &j0, &j1);
                mg_support(K, fnz, cnz, &k0, &k1);
                double zs = 0.0;
                for (int64_t k = k0; k <= k1; k++) {
                    double ys = 0.0;
                    for (int64_t j = j0; j <= j1; j++) {
                        double xs = 0.0;
                        for (int64_t i = i0; i <= i1; i++)
                            xs = xs + (mg_w64(i, I, fnx, cnx) * res[MG_FI(i, j, k)]);
                        ys = ys + (mg_w64(j, J, fny, cny) * xs);
                    }
                    zs = zs + (mg_w64(k, K, fnz, cnz) * ys);
                }
                rc[((K - 1) * cny + (J - 1)) * cnx + (I - 1)] = zs * scale;
            }
}

void oracle_mg_restrict_f32(int64_t fnx, int64_t fny, int64_t fnz, const float *res, float *rc,
                            double scale64)
{
    const float scale = (float)scale64;
    const int64_t cnx = oracle_mg_coarse_n(fnx), cny = oracle_mg_coarse_n(fny),
                  cnz = oracle_mg_coarse_n(fnz);
    for (int64_t K = 1; K <= cnz; K++)
        for (int64_t J = 1; J <= cny; J++)
            for (int64_t I = 1; I <= cnx; I++) {
                int64_t i0, i1, j0, j1, k0, k1;
                mg_support(I, fnx, cnx, &i0, &i1);
                mg_support(J, fny, cny, &j0, &j1);
                mg_support(K, fnz, cnz, &k0, &k1);
                float zs = 0.0f;
                for (int64_t k = k0; k <= k1; k++) {
                    float ys = 0.0f;
                    for (int64_t j = j0; j <= j1; j++) {
                        float xs = 0.0f;
                        for (int64_t i = i0; i <= i1; i++)
                            xs = xs + (mg_w32(i, I, fnx, cnx) * res[MG_FI(i, j, k)]);
                        ys = ys + (mg_w32(j, J, fny, cny) * xs);
                    }
                    zs = zs + (mg_w32(k, K, fnz, cnz) * ys);
                }
                rc[((K - 1) * cny + (J - 1)) * cnx + (I - 1)] = zs * scale;
            }
}

/* e_f += P e_c.  e_f: padded fine grid, ghost width fh; e_c: padded coarse
 * grid, ghost width 1 (ghosts 0). */
void oracle_mg_prolong_add_f64(int64_t fnx, int64_t fny, int64_t fnz, int64_t fh, double *ef,
                               const double *ec)
{
    const int64_t cnx = oracle_mg_coarse_n(fnx), cny = oracle_mg_coarse_n(fny),
                  cnz = oracle_mg_coarse_n(fnz);
    const int64_t fpx = fnx + 2 * fh, fpy = fny + 2 * fh, cpx = cnx + 2, cpy = cny + 2;
    for (int64_t k = 1; k <= fnz; k++)
        for (int64_t j = 1; j <= fny; j++)
            for (int64_t i = 1; i <= fnx; i++) {
                int64_t I0, qi, J0, qj, K0, qk;
                mg_pos(i, fnx, cnx, &I0, &qi);
                mg_pos(j, fny, cny, &J0, &qj);
                mg_pos(k, fnz, cnz, &K0, &qk);
                const double wmx = (double)(fnx + 1 - qi) / (double)(fnx + 1),
                             wqx = (double)qi / (double)(fnx + 1);
                const double wmy = (double)(fny + 1 - qj) / (double)(fny + 1),
                             wqy = (double)qj / (double)(fny + 1);
                const double wmz = (double)(fnz + 1 - qk) / (double)(fnz + 1),
                             wqz = (double)qk / (double)(fnz + 1);
                double vy[2];
                for (int c = 0; c < 2; c++) {
                    double vx[2];
                    for (int b = 0; b < 2; b++) {
                        const double *row = ec + ((K0 + c) * cpy + (J0 + b)) * cpx;
                        vx[b] = (wmx * row[I0]) + (wqx * row[I0 + 1]);
                    }
                    vy[c] = (wmy * vx[0]) + (wqy * vx[1]);
                }
                const double v = (wmz * vy[0]) + (wqz * vy[1]);
                double *p = ef + ((k - 1 + fh) * fpy + (j - 1 + fh)) * fpx + (i - 1 + fh);
                *p = *p + v;
            }
}

void oracle_mg_prolong_add_f32(int64_t fnx, int64_t fny, int64_t fnz, int64_t fh, float *ef,
                               const float *ec)
{
    const int64_t cnx = oracle_mg_coarse_n(fnx), cny = oracle_mg_coarse_n(fny),
                  cnz = oracle_mg_coarse_n(fnz);
    const int64_t fpx = fnx + 2 * fh, fpy = fny + 2 * fh, cpx = cnx + 2, cpy = cny + 2;
    for (int64_t k = 1; k <= fnz; k++)
        for (int64_t j = 1; j <= fny; j++)
            for (int64_t i = 1; i <= fnx; i++) {
                int64_t I0, qi, J0, qj, K0, qk;
                mg_pos(i, fnx, cnx, &I0, &qi);
                mg_pos(j, fny, cny, &J0, &qj);
                mg_pos(k, fnz, cnz, &K0, &qk);
                const float wmx = (float)(fnx + 1 - qi) / (float)(fnx + 1),
                            wqx = (float)qi / (float)(fnx + 1);
                const float wmy = (float)(fny + 1 - qj) / (float)(fny + 1),
                            wqy = (float)qj / (float)(fny + 1);
                const float wmz = (float)(fnz + 1 - qk) / (float)(fnz + 1),
                            wqz = (float)qk / (float)(fnz + 1);
                float vy[2];
                for (int c = 0; c < 2; c++) {
                    float vx[2];
                    for (int b = 0; b < 2; b++) {
                        const float *row = ec + ((K0 + c) * cpy + (J0 + b)) * cpx;
                        vx[b] = (wmx * row[I0]) + (wqx * row[I0 + 1]);
                    }
                    vy[c] = (wmy * vx[0]) + (wqy * vx[1]);
                }
                const float v = (wmz * vy[0]) + (wqz * vy[1]);
                float *p = ef + ((k - 1 + fh) * fpy + (j - 1 + fh)) * fpx + (i - 1 + fh);
                *p = *p + v;
            }
}

/* res = r - ((6*c) - s) for the correction e (padded, ghost width h) and the
 * interior-only right-hand side r; float arithmetic. */
void oracle_mg_residual_f32(int64_t nx, int64_t ny, int64_t nz, int64_t h, const float *u,
                            const float *fp, float *res)
{
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    for (int64_t k = h; k < h + nz; k++)
        for (int64_t j = h; j < h + ny; j++)
            for (int64_t i = h; i < h + nx; i++) {
                float s = u[IDX(k, j, i - 1)];
                s = s + u[IDX(k, j, i + 1)];
                s = s + u[IDX(k, j - 1, i)];
                s = s + u[IDX(k, j + 1, i)];
                s = s + u[IDX(k - 1, j, i)];
                s = s + u[IDX(k + 1, j, i)];
                const float c = u[IDX(k, j, i)];
                res[FIDX(k, j, i)] = fp[FIDX(k, j, i)] - ((6.0f * c) - s);
            }
}

typedef struct {
    int64_t nx, ny, nz, h;
    void *e, *r, *res; /* padded correction; interior-only rhs and residual */
} mg_level;

static void mg_smooth(int smoother, int f32, const mg_level *L, int sweeps)
{
    if (sweeps <= 0) return;
    const double w = smoother == 0 ? 1.0 / 7.0 : 1.0 / 6.0;
    const double a = smoother == 0 ? 1.0 / 7.0 : 0.0;
    if (f32) {
        if (smoother == 0)
            oracle_jacobi_f32(L->nx, L->ny, L->nz, L->h, L->e, L->r, a, w, w, sweeps);
        else if (smoother == 1)
            oracle_gs_f32(L->nx, L->ny, L->nz, L->h, L->e, L->r, a, w, w, sweeps);
        else
            oracle_rbgs_f32(L->nx, L->ny, L->nz, L->h, L->e, L->r, a, w, w, sweeps);
    } else {
        if (smoother == 0)
            oracle_jacobi_f64(L->nx, L->ny, L->nz, L->h, L->e, L->r, a, w, w, sweeps);
        else if (smoother == 1)
            oracle_gs_f64(L->nx, L->ny, L->nz, L->h, L->e, L->r, a, w, w, sweeps);
        else
            oracle_rbgs_f64(L->nx, L->ny, L->nz, L->h, L->e, L->r, a, w, w, sweeps);
    }
}

static void mg_vcycle(mg_level *lv, int l, int nlev, int smoother, int f32, int pre, int post,
                      int coarse)
{
    mg_level *L = &lv[l];
    const size_t es = f32 ? sizeof(float) : sizeof(double);
    const int64_t n = (L->nx + 2 * L->h) * (L->ny + 2 * L->h) * (L->nz + 2 * L->h);
    memset(L->e, 0, (size_t)n * es);
    if (l == nlev - 1) {
        mg_smooth(smoother, f32, L, coarse);
        return;
    }
    mg_smooth(smoother, f32, L, pre);
    mg_level *C = &lv[l + 1];
    const double scale = oracle_mg_scale(L->nx, L->ny, L->nz);
    if (f32) {
        oracle_mg_residual_f32(L->nx, L->ny, L->nz, L->h, L->e, L->r, L->res);
        oracle_mg_restrict_f32(L->nx, L->ny, L->nz, L->res, C->r, scale);
    } else {
        oracle_residual_f64(L->nx, L->ny, L->nz, L->h, L->e, L->r, L->res);
        oracle_mg_restrict_f64(L->nx, L->ny, L->nz, L->res, C->r, scale);
    }
    mg_vcycle(lv, l + 1, nlev, smoother, f32, pre, post, coarse);
    if (f32)
        oracle_mg_prolong_add_f32(L->nx, L->ny, L->nz, L->h, L->e, C->e);
    else
        oracle_mg_prolong_add_f64(L->nx, L->ny, L->nz, L->h, L->e, C->e);
    mg_smooth(smoother, f32, L, post);
}

/* Number of levels of a grid (coarsening while every axis has >= 3 points). */
int oracle_mg_levels(int64_t nx, int64_t ny, int64_t nz)
{
    int n = 1;
    while (nx >= 3 && ny >= 3 && nz >= 3 && n < 32) {
        nx = oracle_mg_coarse_n(nx);
        ny = oracle_mg_coarse_n(ny);
        nz = oracle_mg_coarse_n(nz);
        n++;
    }
    return n;
}

/* Multigrid-preconditioned defect correction: returns 0 on convergence, -6
 * when max_cycles V-cycles were applied without reaching tol, -2 when out of
 * memory.  *cycles_done = V-cycles applied; *rel_out = last ||r|| / ||f'||;
 * rel_hist (may be NULL; max_cycles + 1 entries) receives every relative
 * residual. */
int oracle_mg_solve(int64_t nx, int64_t ny, int64_t nz, int64_t h, int smoother, int inner_f32,
                    double *u, const double *fp, int pre, int post, int coarse, double tol,
                    int max_cycles, int *cycles_done, double *rel_out, double *rel_hist)
{
    const int nlev = oracle_mg_levels(nx, ny, nz);
    mg_level lv[32];
    const size_t es = inner_f32 ? sizeof(float) : sizeof(double);
    int ok = 1;
    for (int l = 0; l < nlev; l++) {
        mg_level *L = &lv[l];
        if (l == 0) {
            L->nx = nx; L->ny = ny; L->nz = nz; L->h = h;
        } else {
            L->nx = oracle_mg_coarse_n(lv[l - 1].nx);
            L->ny = oracle_mg_coarse_n(lv[l - 1].ny);
            L->nz = oracle_mg_coarse_n(lv[l - 1].nz);
            L->h = 1;
        }
        const int64_t n = (L->nx + 2 * L->h) * (L->ny + 2 * L->h) * (L->nz + 2 * L->h);
        const int64_t nil = L->nx * L->ny * L->nz;
        L->e = calloc((size_t)n, es);
        L->r = calloc((size_t)nil, es);
        L->res = calloc((size_t)nil, es);
        if (!L->e || !L->r || !L->res) ok = 0;
    }
    const int64_t ni = nx * ny * nz;
    const int64_t px = nx + 2 * h, py = ny + 2 * h;
    double *r = (double *)malloc((size_t)ni * sizeof(double));
    int status = ok && r ? -6 : -2, cyc = 0;
    double rel = INFINITY;
    if (status == -6) {
        const double nf = sqrt(oracle_sumsq(fp, ni));
        for (;;) {
            rel = sqrt(oracle_residual_f64(nx, ny, nz, h, u, fp, r)) / nf;
            if (rel_hist) rel_hist[cyc] = rel;
            if (rel <= tol) { status = 0; break; }
            if (cyc >= max_cycles) break;
            if (inner_f32)
                for (int64_t q = 0; q < ni; q++) ((float *)lv[0].r)[q] = (float)r[q];
            else
                memcpy(lv[0].r, r, (size_t)ni * sizeof(double));
            mg_vcycle(lv, 0, nlev, smoother, inner_f32, pre, post, coarse);
            for (int64_t k = h; k < h + nz; k++)
                for (int64_t j = h; j < h + ny; j++)
                    for (int64_t i = h; i < h + nx; i++)
                        u[IDX(k, j, i)] = u[IDX(k, j, i)] +
                                          (inner_f32 ? (double)((float *)lv[0].e)[IDX(k, j, i)]
                                                     : ((double *)lv[0].e)[IDX(k, j, i)]);
            cyc++;
        }
    }
    for (int l = 0; l < nlev; l++) { free(lv[l].e); free(lv[l].r); free(lv[l].res); }
    free(r);
    if (cycles_done) *cycles_done = cyc;
    if (rel_out) *rel_out = rel;
    return status;
}
