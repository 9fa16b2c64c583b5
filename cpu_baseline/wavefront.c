/*
 * wavefront.c -- the paper's own multicore schemes on the host CPU, as a
 * paper-comparable CPU baseline next to the GPU library (FP64, POSIX threads).
 *
 *   wf_jacobi_f64: temporal wavefront blocking (Sec. 4).  A thread group of t
 *       threads updates one y-block; thread tau performs sweep tau and walks
 *       the planes in z two planes behind thread tau-1 (the paper's "distance
 *       of two"), so the planes a thread reads were finished by its
 *       predecessor one step earlier and are still in the shared cache.  All
 *       threads meet in a spin barrier after every plane step.  Intermediate
 *       levels live in a small round-robin plane ring per level (four planes
 *       of the block's rows); only the last level is written to the output
 *       grid.  The y-blocks are skewed (level tau of block b covers rows
 *       [a_b - tau, a_{b+1} - tau)) so that a block depends only on the block
 *       before it, through a boundary array that keeps the last two rows of
 *       every intermediate level for all planes: no site is computed twice.
 *       Several thread groups update consecutive blocks at the same time, in
 *       lockstep (one barrier for all threads).
 *   wf_gs_f64: pipeline-parallel lexicographic Gauss-Seidel (Sec. 3) combined
 *       with the temporal wavefront (Sec. 4).  The rows of a plane are split
 *       into P sub-blocks; thread (tau, p) performs sweep tau on sub-block p
 *       of plane k at step k + p + 2*tau, so every fresh neighbour (x-, y-,
 *       z-) of a site was written in an earlier step and every old one (x+,
 *       y+, z+) was finished by the previous sweep and not yet overwritten:
 *       the result is that of the sequential loop nest.  With t = 1 this is
 *       the plain pipeline-parallel baseline of Sec. 3.
 *
 * Both give bit-identical results to the plain loop nests: every site value
 * is computed once per sweep with the Sec. 3 operand order
 *     s = ((((x- + x+) + y-) + y+) + z-) + z+,  v = (a*c) + (b*s) [+ g*f]
 * (the a*c term omitted when a == 0), with FP contraction off.  Only the
 * order in which independent sites are computed changes.
 *
 * Grid layout: interior nx, ny, nz and a ghost layer of width h >= 1; a C
 * array of (nz+2h)(ny+2h)(nx+2h) doubles, x contiguous; f (optional) is
 * interior-only, nz*ny*nx values.
 *
 * Build: gcc -O3 -march=x86-64-v3 -ffp-contract=off -fno-fast-math -pthread -shared -fPIC
 * (AVX2 vectors; contraction off, so every element sees the same operations)
 */
#define _GNU_SOURCE
#include <pthread.h>
#include <sched.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#if defined(__x86_64__) || defined(__i386__)
#include <immintrin.h>
#define CPU_RELAX() _mm_pause()
#else
#define CPU_RELAX() ((void)0)
#endif

/* ------------------------------------------------------------ barrier ---- */

/* Centralised sense-reversing spin barrier.  A waiter spins on the shared
 * sense flag and yields the core after a while, so an oversubscribed machine
 * still makes progress. */
typedef struct {
    _Atomic int count;
    _Atomic int sense;
    int n;
} spin_barrier;

static void barrier_init(spin_barrier *b, int n)
{
    atomic_store(&b->count, n);
    atomic_store(&b->sense, 0);
    b->n = n;
}

static void barrier_wait(spin_barrier *b, int *local_sense)
{
    const int s = !*local_sense;
    *local_sense = s;
    if (atomic_fetch_sub_explicit(&b->count, 1, memory_order_acq_rel) == 1) {
        atomic_store_explicit(&b->count, b->n, memory_order_relaxed);
        atomic_store_explicit(&b->sense, s, memory_order_release);
        return;
    }
    int spins = 0;
    while (atomic_load_explicit(&b->sense, memory_order_acquire) != s) {
        if (++spins < 2048) {
            CPU_RELAX();
        } else {
            sched_yield();
            spins = 0;
        }
    }
}

/* Start gate of a team of threads: every worker waits on it before doing
 * anything, and the launcher opens it (1) once all threads exist.  If a
 * thread cannot be created, the gate is set to abort (-1) instead and the
 * workers already started return at once, so none of them waits in a
 * barrier that could never fill. */
static int wait_gate(_Atomic int *gate)
{
    int g, spins = 0;
    while ((g = atomic_load_explicit(gate, memory_order_acquire)) == 0) {
        if (++spins < 2048) {
            CPU_RELAX();
        } else {
            sched_yield();
            spins = 0;
        }
    }
    return g > 0;
}

static int run_threads(int n, void *(*fn)(void *), void *args, size_t argsz, _Atomic int *gate)
{
    pthread_t *tid = (pthread_t *)malloc((size_t)n * sizeof(pthread_t));
    if (!tid) return -2;
    atomic_store(gate, 0);
    int started = 0, rc = 0;
    for (; started < n; started++)
        if (pthread_create(&tid[started], NULL, fn, (char *)args + (size_t)started * argsz)) {
            rc = -3;
            break;
        }
    atomic_store_explicit(gate, rc == 0 ? 1 : -1, memory_order_release);
    for (int i = 0; i < started; i++) pthread_join(tid[i], NULL);
    free(tid);
    return rc;
}

/* --------------------------------------------------------- row update ---- */

/* One row of sites i = h .. h+nx-1 of a Jacobi level: c is the row of the
 * level below at the same (y, z), ym/yp/zm/zp its neighbour rows, out the
 * destination row (all indexed by padded x). */
static inline void jacobi_row(int64_t h, int64_t nx, const double *restrict c,
                              const double *restrict ym, const double *restrict yp,
                              const double *restrict zm, const double *restrict zp,
                              const double *restrict f, double a, double b, double g,
                              double *restrict out)
{
    if (a != 0.0) {
        if (f) {
            for (int64_t i = h; i < h + nx; i++) {
                double s = c[i - 1] + c[i + 1];
                s = s + ym[i];
                s = s + yp[i];
                s = s + zm[i];
                s = s + zp[i];
                double v = (a * c[i]) + (b * s);
                out[i] = v + (g * f[i - h]);
            }
        } else {
            for (int64_t i = h; i < h + nx; i++) {
                double s = c[i - 1] + c[i + 1];
                s = s + ym[i];
                s = s + yp[i];
                s = s + zm[i];
                s = s + zp[i];
                out[i] = (a * c[i]) + (b * s);
            }
        }
    } else {
        if (f) {
            for (int64_t i = h; i < h + nx; i++) {
                double s = c[i - 1] + c[i + 1];
                s = s + ym[i];
                s = s + yp[i];
                s = s + zm[i];
                s = s + zp[i];
                out[i] = (b * s) + (g * f[i - h]);
            }
        } else {
            for (int64_t i = h; i < h + nx; i++) {
                double s = c[i - 1] + c[i + 1];
                s = s + ym[i];
                s = s + yp[i];
                s = s + zm[i];
                s = s + zp[i];
                out[i] = b * s;
            }
        }
    }
}

/* One row of an in-place Gauss-Seidel sweep: r is the row being updated
 * (x- is the value just written), ym/zm hold this sweep's values, yp/zp the
 * previous sweep's. */
static inline void gs_row(int64_t h, int64_t nx, double *restrict r, const double *restrict ym,
                          const double *restrict yp, const double *restrict zm,
                          const double *restrict zp, const double *restrict f, double a,
                          double b, double g)
{
    double xm = r[h - 1];
    for (int64_t i = h; i < h + nx; i++) {
        double s = xm + r[i + 1];
        s = s + ym[i];
        s = s + yp[i];
        s = s + zm[i];
        s = s + zp[i];
        double v;
        if (a != 0.0)
            v = (a * r[i]) + (b * s);
        else
            v = b * s;
        if (f) v = v + (g * f[i - h]);
        r[i] = v;
        xm = v;
    }
}

/* ------------------------------------------- Jacobi temporal wavefront ---- */

#define RING 4 /* planes per intermediate level: z-1, z, z+1 and the one being written */

typedef struct {
    int64_t nx, ny, nz, h, px, py;
    const double *src; /* level 0 of this pass */
    double *dst;       /* level `levels` of this pass (ghosts already set) */
    const double *f;
    double a, b, g;
    int levels;        /* sweeps of this pass (<= t) */
    int t, groups;
    int nblocks;
    const int64_t *ablk;   /* block starts a_0..a_nblocks (padded rows) */
    int64_t ring_rows;     /* rows per ring plane */
    double **ring;         /* [group][level 1..t-1][RING] planes of ring_rows * px */
    double **bnd;          /* [slot][level 1..t-1] nz * 2 rows of px */
    int nslots;
    spin_barrier bar;
    _Atomic int gate;
} jac_ctx;

typedef struct {
    jac_ctx *c;
    int grp, tau; /* tau = 1..t */
} jac_thread;

/* rows [lo, hi) of level l in block b (padded coordinates) */
static inline void level_rows(const jac_ctx *c, int b, int l, int64_t *lo, int64_t *hi)
{
    const int64_t top = c->h + c->ny;
    *lo = b == 0 ? c->h : c->ablk[b] - l;
    *hi = b == c->nblocks - 1 ? top : c->ablk[b + 1] - l;
}

static inline double *ring_plane(const jac_ctx *c, int grp, int l, int64_t q)
{
    return c->ring[((int64_t)grp * (c->t - 1) + (l - 1)) * RING + (q % RING)];
}

static inline double *bnd_rows(const jac_ctx *c, int slot, int l, int64_t q)
{
    return c->bnd[(int64_t)slot * (c->t - 1) + (l - 1)] + ((q - c->h) * 2) * c->px;
}

/* Row y of level l at plane q, as seen by block b of group grp. */
static inline const double *level_row(const jac_ctx *c, int grp, int b, int l, int64_t q,
                                      int64_t y)
{
    const int64_t h = c->h;
    if (l == 0 || q < h || q >= h + c->nz || y < h || y >= h + c->ny)
        return c->src + (q * c->py + y) * c->px; /* level 0, or a ghost (same at every level) */
    int64_t lo, hi;
    level_rows(c, b, l, &lo, &hi);
    if (y < lo) /* one of the two rows kept by the block before */
        return bnd_rows(c, (b - 1) % c->nslots, l, q) + (y - (lo - 2)) * c->px;
    return ring_plane(c, grp, l, q) + (y - lo) * c->px;
}

static void *jac_worker(void *arg)
{
    jac_thread *th = (jac_thread *)arg;
    jac_ctx *c = th->c;
    const int tau = th->tau, grp = th->grp;
    const int64_t h = c->h, nx = c->nx, px = c->px;
    const int64_t nsteps = c->nz + 2 * (c->t - 1);
    const int rounds = (c->nblocks + c->groups - 1) / c->groups;
    int sense = 0;
    if (!wait_gate(&c->gate)) return NULL;
    for (int rd = 0; rd < rounds; rd++) {
        const int b = rd * c->groups + grp;
        const int active = b < c->nblocks && tau <= c->levels;
        int64_t lo = 0, hi = 0;
        if (active) level_rows(c, b, tau, &lo, &hi);
        for (int64_t s = 0; s < nsteps; s++) {
            const int64_t q = h + s - 2 * (tau - 1); /* plane of this thread's level */
            if (active && q >= h && q < h + c->nz) {
                const int last = tau == c->levels;
                for (int64_t y = lo; y < hi; y++) {
                    const double *cc = level_row(c, grp, b, tau - 1, q, y);
                    const double *ym = level_row(c, grp, b, tau - 1, q, y - 1);
                    const double *yp = level_row(c, grp, b, tau - 1, q, y + 1);
                    const double *zm = level_row(c, grp, b, tau - 1, q - 1, y);
                    const double *zp = level_row(c, grp, b, tau - 1, q + 1, y);
                    const double *fr = c->f ? c->f + ((q - h) * c->ny + (y - h)) * nx : NULL;
                    double *out;
                    if (last) {
                        out = c->dst + (q * c->py + y) * px;
                    } else {
                        out = ring_plane(c, grp, tau, q) + (y - lo) * px;
                        out[h - 1] = cc[h - 1]; /* x ghosts of this row */
                        out[h + nx] = cc[h + nx];
                    }
                    jacobi_row(h, nx, cc, ym, yp, zm, zp, fr, c->a, c->b, c->g, out);
                }
                /* the next block reads the last two rows of this level */
                if (!last && b + 1 < c->nblocks) {
                    double *bd = bnd_rows(c, b % c->nslots, tau, q);
                    memcpy(bd, ring_plane(c, grp, tau, q) + (hi - 2 - lo) * px,
                           (size_t)(2 * px) * sizeof(double));
                }
            }
            barrier_wait(&c->bar, &sense);
        }
    }
    return NULL;
}


/* Plan of the y-blocks: nblocks blocks of about block_y rows; every block but
 * the last needs at least t + 2 rows so that the two kept rows of each level
 * belong to it.  Returns the block count; starts in ablk[0..n]. */
static int plan_blocks(int64_t h, int64_t ny, int t, int64_t block_y, int64_t *ablk, int maxb)
{
    if (block_y < t + 2) block_y = t + 2;
    int n = (int)(ny / block_y);
    if (n < 1) n = 1;
    if (n > maxb) n = maxb;
    for (int i = 0; i < n; i++) ablk[i] = h + (ny * i) / n;
    ablk[n] = h + ny;
    for (int i = 0; i + 1 < n; i++)
        if (ablk[i + 1] - ablk[i] < t + 2) return plan_blocks(h, ny, t, block_y + 1, ablk, n - 1);
    return n;
}

/*
 * `sweeps` Jacobi sweeps; result in u.  scratch: a second grid of the same
 * size (its ghosts are set here).  t: sweeps per wavefront pass (threads per
 * group, 1..16); groups: thread groups (1..64); block_y: rows per y-block.
 * Returns 0, -1 on bad arguments, -2 if out of memory, -3 if threads could
 * not be started.
 */
int wf_jacobi_f64(int64_t nx, int64_t ny, int64_t nz, int64_t h, double *u, double *scratch,
                  const double *f, double a, double b, double g, int sweeps, int t, int groups,
                  int64_t block_y)
{
    if (nx < 1 || ny < 1 || nz < 1 || h < 1 || sweeps < 0 || t < 1 || t > 16 || groups < 1 ||
        groups > 64 || !u || !scratch)
        return -1;
    if (sweeps == 0) return 0;
    const int64_t px = nx + 2 * h, py = ny + 2 * h, pz = nz + 2 * h;
    memcpy(scratch, u, (size_t)(px * py * pz) * sizeof(double)); /* identical ghosts */

    int64_t ablk[4097];
    const int nblocks = plan_blocks(h, ny, t, block_y, ablk, 4096);
    if (groups > nblocks) groups = nblocks;
    int64_t maxrows = 0;
    for (int i = 0; i < nblocks; i++)
        if (ablk[i + 1] - ablk[i] > maxrows) maxrows = ablk[i + 1] - ablk[i];
    const int64_t ring_rows = maxrows + t; /* the last block's levels reach t rows lower */
    const int nslots = groups + 1;

    jac_ctx c;
    memset(&c, 0, sizeof(c));
    c.nx = nx; c.ny = ny; c.nz = nz; c.h = h; c.px = px; c.py = py;
    c.f = f; c.a = a; c.b = b; c.g = g;
    c.t = t; c.groups = groups; c.nblocks = nblocks; c.ablk = ablk;
    c.ring_rows = ring_rows; c.nslots = nslots;
    const int nl = t > 1 ? t - 1 : 0;
    const int nring = groups * nl * RING, nbnd = nslots * nl;
    c.ring = (double **)calloc((size_t)(nring + 1), sizeof(double *));
    c.bnd = (double **)calloc((size_t)(nbnd + 1), sizeof(double *));
    jac_thread *th = (jac_thread *)malloc((size_t)(groups * t) * sizeof(jac_thread));
    int rc = (c.ring && c.bnd && th) ? 0 : -2;
    for (int i = 0; rc == 0 && i < nring; i++)
        if (!(c.ring[i] = (double *)malloc((size_t)(ring_rows * px) * sizeof(double)))) rc = -2;
    for (int i = 0; rc == 0 && i < nbnd; i++)
        if (!(c.bnd[i] = (double *)malloc((size_t)(nz * 2 * px) * sizeof(double)))) rc = -2;

    double *A = u, *B = scratch;
    int done = 0;
    while (rc == 0 && done < sweeps) {
        c.levels = sweeps - done < t ? sweeps - done : t;
        c.src = A;
        c.dst = B;
        barrier_init(&c.bar, groups * t);
        for (int gi = 0; gi < groups; gi++)
            for (int ti = 0; ti < t; ti++) {
                th[gi * t + ti].c = &c;
                th[gi * t + ti].grp = gi;
                th[gi * t + ti].tau = ti + 1;
            }
        rc = run_threads(groups * t, jac_worker, th, sizeof(jac_thread), &c.gate);
        done += c.levels;
        double *tmp = A;
        A = B;
        B = tmp;
    }
    if (rc == 0 && A != u) memcpy(u, A, (size_t)(px * py * pz) * sizeof(double));
    for (int i = 0; c.ring && i < nring; i++) free(c.ring[i]);
    for (int i = 0; c.bnd && i < nbnd; i++) free(c.bnd[i]);
    free(c.ring);
    free(c.bnd);
    free(th);
    return rc;
}

/* ----------------------------------- pipeline-parallel Gauss-Seidel ---- */

typedef struct {
    int64_t nx, ny, nz, h, px, py;
    double *u;
    const double *f;
    double a, b, g;
    int t, P, levels;
    const int64_t *jb; /* sub-block row starts jb[0..P] */
    spin_barrier bar;
    _Atomic int gate;
} gs_ctx;

typedef struct {
    gs_ctx *c;
    int tau, p; /* sweep within the group (0..t-1), sub-block (0..P-1) */
} gs_thread;

static void *gs_worker(void *arg)
{
    gs_thread *th = (gs_thread *)arg;
    gs_ctx *c = th->c;
    const int64_t h = c->h, nx = c->nx, px = c->px, py = c->py;
    const int64_t nsteps = c->nz + (c->P - 1) + 2 * (c->t - 1);
    const int active = th->tau < c->levels;
    int sense = 0;
    if (!wait_gate(&c->gate)) return NULL;
    for (int64_t s = 0; s < nsteps; s++) {
        const int64_t k = h + s - th->p - 2 * th->tau;
        if (active && k >= h && k < h + c->nz) {
            for (int64_t j = c->jb[th->p]; j < c->jb[th->p + 1]; j++) {
                double *r = c->u + (k * py + j) * px;
                const double *fr = c->f ? c->f + ((k - h) * c->ny + (j - h)) * nx : NULL;
                gs_row(h, nx, r, r - px, r + px, r - px * py, r + px * py, fr, c->a, c->b,
                       c->g);
            }
        }
        barrier_wait(&c->bar, &sense);
    }
    return NULL;
}

/*
 * `sweeps` lexicographic Gauss-Seidel sweeps in place on u.  t: sweeps in
 * flight (1..16; 1 = the pipeline-parallel baseline); P: sub-blocks per plane
 * (1..256; clamped to ny).  t * P threads.  Returns 0, -1 on bad arguments,
 * -2 if out of memory, -3 if threads could not be started.
 */
int wf_gs_f64(int64_t nx, int64_t ny, int64_t nz, int64_t h, double *u, const double *f,
              double a, double b, double g, int sweeps, int t, int P)
{
    if (nx < 1 || ny < 1 || nz < 1 || h < 1 || sweeps < 0 || t < 1 || t > 16 || P < 1 ||
        P > 256 || !u)
        return -1;
    if (sweeps == 0) return 0;
    if (P > ny) P = (int)ny;
    int64_t jb[257];
    for (int i = 0; i <= P; i++) jb[i] = h + (ny * i) / P;
    gs_ctx c;
    memset(&c, 0, sizeof(c));
    c.nx = nx; c.ny = ny; c.nz = nz; c.h = h; c.px = nx + 2 * h; c.py = ny + 2 * h;
    c.u = u; c.f = f; c.a = a; c.b = b; c.g = g;
    c.t = t; c.P = P; c.jb = jb;
    gs_thread *th = (gs_thread *)malloc((size_t)(t * P) * sizeof(gs_thread));
    if (!th) return -2;
    int rc = 0, done = 0;
    while (rc == 0 && done < sweeps) {
        c.levels = sweeps - done < t ? sweeps - done : t;
        barrier_init(&c.bar, t * P);
        for (int ti = 0; ti < t; ti++)
            for (int p = 0; p < P; p++) {
                th[ti * P + p].c = &c;
                th[ti * P + p].tau = ti;
                th[ti * P + p].p = p;
            }
        rc = run_threads(t * P, gs_worker, th, sizeof(gs_thread), &c.gate);
        done += c.levels;
    }
    free(th);
    return rc;
}

/* Threads this process may run on (its CPU affinity set). */
int wf_cpu_count(void)
{
    cpu_set_t cs;
    if (sched_getaffinity(0, sizeof(cs), &cs) != 0) return 1;
    const int n = CPU_COUNT(&cs);
    return n > 0 ? n : 1;
}
