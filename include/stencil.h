/*
 * stencil.h -- C ABI of libstencil, an MI355X (gfx950) library of iterated
 * 3D 7-point smoothers: two-array Jacobi and in-place lexicographic
 * Gauss-Seidel with several sweeps fused per pass over HBM, an FP64
 * iterative-refinement solve around an FP32 inner smoother, and a
 * continuous-batching job service.
 *
 * The methods are those of Treibig, Wellein, Hager, "Efficient
 * multicore-aware parallelization strategies for iterative stencil
 * computations" (Sec. 3 defines the Jacobi and Gauss-Seidel loop nests,
 * Sec. 4 the temporal wavefront blocking; Eq. (1) the bandwidth model).
 *
 * ---------------------------------------------------------------------------
 * Common conventions
 *
 *  Grid layout.  A grid has interior extents nx, ny, nz >= 1 and a ghost
 *  layer of width halo >= 1 on every side.  It is one dense C array of
 *  (nz+2*halo)*(ny+2*halo)*(nx+2*halo) elements, x contiguous:
 *      index(k, j, i) = (k*(ny+2*halo) + j)*(nx+2*halo) + i,
 *  interior i in [halo, halo+nx), likewise j, k.  Ghost cells hold Dirichlet
 *  values; they are read (the innermost layer only) and never written by a
 *  sweep.  A right-hand side f is interior-only: nz*ny*nx elements, x
 *  contiguous.  The Sec. 3 listings read i-1 and i+1 at every interior site,
 *  which implies this ghost layer.
 *
 *  Site update (Sec. 3 loop nests, with the Poisson right-hand side the
 *  paper names; C left-to-right association of the printed sum):
 *      s = ((((x- + x+) + y-) + y+) + z-) + z+
 *      v = (center*c) + (neighbor*s)     -- center*c omitted when center == 0
 *      v = v + (rhs*f)                   -- only when f != NULL
 *  No fused multiply-add is used anywhere, so FP64 (and FP32) results are
 *  bit-identical to a sequential CPU evaluation in the same order.  Jacobi
 *  reads all operands from the previous sweep; Gauss-Seidel is in place in
 *  lexicographic order (i fastest, then j, then k), so x-, y-, z- are new and
 *  x+, y+, z+ are old.  Equal results are compared by value (+0 == -0).
 *
 *  dtype: ST_FP64 (double) or ST_FP32 (float storage and float arithmetic;
 *  weights are rounded to float once).
 *
 *  Memory.  Every grid pointer is a device pointer (hipMalloc'd or a torch
 *  device tensor).  The caller owns u, scratch and f; the library never frees
 *  them and keeps no pointer after the stream work completes.  The library
 *  owns only its internal flag/queue/workspace buffers.
 *
 *  Streams.  hip_stream is a hipStream_t (NULL = the default stream).
 *  stencil_jacobi and stencil_gs only enqueue work and return; results are
 *  ready when the stream reaches that point.
 *
 *  Errors.  Every function returns an st_status (0 or negative).  Argument
 *  errors are detected before anything is enqueued.  A HIP launch failure is
 *  ST_EHIP.  stencil_last_error() returns a thread-local message for the most
 *  recent failure on the calling thread.  No C++ exception crosses the ABI.
 * ---------------------------------------------------------------------------
 */
#ifndef STENCIL_H
#define STENCIL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ST_OK = 0,
    ST_EINVAL = -1,     /* invalid argument (dims, halo, dtype, pointer, t_fuse, ...) */
    ST_ENOMEM = -2,     /* device or host allocation failed / budget too small */
    ST_EHIP = -3,       /* a HIP runtime call or kernel launch failed */
    ST_EBUSY = -4,      /* resource in use (e.g. service shutting down) */
    ST_ENOENT = -5,     /* unknown job id */
    ST_ENOCONV = -6,    /* refinement stopped at max_outer above rel_tol */
    ST_ECANCELED = -7   /* job was cancelled */
} st_status;

typedef enum { ST_FP64 = 0, ST_FP32 = 1 } st_dtype;

typedef enum { ST_BC_KEEP = 0, ST_BC_CONST = 1 } st_bc;

/* Interior extents (>= 1) and ghost width (1..4096).  One padded plane,
 * (nx + 2*halo) * (ny + 2*halo) elements, must span < 2^31 bytes at 8 bytes
 * per element (< 2^28 elements): kernels address a plane with 32-bit byte
 * offsets.  Larger grids are ST_EINVAL. */
typedef struct {
    int64_t nx, ny, nz;
    int32_t halo;
} st_grid;

/* v = (center*c) + (neighbor*s) [+ rhs*f]; the paper's Jacobi uses
 * center = a, neighbor = b; its Gauss-Seidel has center = 0. */
typedef struct {
    double center, neighbor, rhs;
} st_weights;

/*
 * stencil_jacobi -- `sweeps` two-array Jacobi sweeps (Sec. 3 loop nest),
 * fused `t` at a time per pass over HBM (Sec. 4 temporal wavefront blocking,
 * re-expressed as a z-marching GPU tile that keeps the t time levels on chip).
 *
 *  u        in/out grid (dtype), result returned in u.
 *  scratch  second grid of the same size (dtype); its contents on entry are
 *           ignored and on return are unspecified.  Must not alias u.
 *  f        interior-only right-hand side (dtype) or NULL.
 *  w        weights (see above); w->rhs is ignored when f == NULL.
 *  bc       ST_BC_KEEP: use u's ghost cells as given; ST_BC_CONST: first set
 *           every ghost cell of u to bc_value.
 *  sweeps   >= 0 (0 only applies bc).
 *  t_fuse   sweeps fused per pass: 0 = automatic, or 1..8, or 16.  A pass
 *           keeps at most 8 levels on chip; 16 runs as passes of 8.  Any
 *           other value is ST_EINVAL.
 *  Result: bit-identical to `sweeps` sequential sweeps for every t_fuse.
 */
int stencil_jacobi(const st_grid *grid, int32_t dtype, void *u, void *scratch, const void *f,
                   const st_weights *w, int32_t bc, double bc_value, int32_t sweeps,
                   int32_t t_fuse, void *hip_stream);

/*
 * stencil_jacobi_plan -- the pass schedule stencil_jacobi uses for
 * (dtype, f != NULL, sweeps, t_fuse): writes the number of kernel launches to
 * *passes, up to max_list per-pass fused-sweep counts to t_list (may be
 * NULL), and whether a final scratch->u copy is needed to *final_copy (may be
 * NULL).  has_rhs: nonzero when stencil_jacobi gets a right-hand side (the
 * automatic depth differs).  Host-only; ST_EINVAL for a bad dtype, sweeps or
 * t_fuse, or passes == NULL.
 */
int stencil_jacobi_plan(int32_t dtype, int32_t has_rhs, int32_t sweeps, int32_t t_fuse,
                        int32_t *passes, int32_t *t_list, int32_t max_list, int32_t *final_copy);

/*
 * stencil_jacobi_tiles -- how one fused pass of `levels` time levels (1..8)
 * tiles the x-y cross-section of a grid: stencil_jacobi runs t_fuse sweeps
 * as t_fuse levels, stencil_rbgs one red-black sweep as two levels.  Writes
 * the stored tile width and height (each tile also reads `levels` sites
 * beyond them on every side: the dependency cone of Sec. 4's temporal
 * blocking), the number of x-y tiles, and how many of them lie wholly inside
 * the interior (those run without per-site boundary masks).  Host-only; any
 * output pointer may be NULL.  ST_EINVAL for a bad grid, dtype or level count.
 */
int stencil_jacobi_tiles(const st_grid *grid, int32_t dtype, int32_t has_rhs, int32_t levels,
                         int32_t *tile_w, int32_t *tile_h, int32_t *tiles, int32_t *interior);

/*
 * stencil_gs -- `sweeps` in-place lexicographic Gauss-Seidel sweeps
 * (Sec. 3 loop nest), run as a pipelined wavefront: the pipeline-parallel
 * and temporal-wavefront schemes of Sec. 3/4 re-expressed as bundles of
 * x-lines scheduled in topological order with per-bundle progress counters
 * instead of barriers.  t_fuse sweeps are in flight per launch (0 = all
 * sweeps in one launch, at most 4095; 1 = one launch per sweep; 1..8 or 16
 * accepted).  Bit-identical to the sequential loop nest.  Each launch takes
 * its workspace (progress counters, ticket and item table, about 8 bytes per
 * (sweep, 8x8 bundle of x-lines)) from the stream-ordered allocator
 * (hipMallocAsync on hip_stream) and returns it after the launch; waits are
 * bounded (see stencil_sync).
 * Same argument meanings as stencil_jacobi.
 */
int stencil_gs(const st_grid *grid, int32_t dtype, void *u, const void *f, const st_weights *w,
               int32_t bc, double bc_value, int32_t sweeps, int32_t t_fuse, void *hip_stream);

/*
 * stencil_gs_noalloc -- stencil_gs for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same sweeps, arguments, result bits and bounded
 * waits, but no hipMalloc, hipMallocAsync, hipFree or other allocating call.
 * The wavefront workspace (progress counters, ticket, item table) lives in a
 * static device array of 4 MiB that the library holds on every device it
 * runs on until the process ends.  Each launch clears what it uses, so no
 * state carries over between calls; calls that overlap on one device (on
 * different streams, or from different threads) race for the array and must
 * not be issued.  One launch needs about 8 bytes per (sweep, 8x8 bundle of
 * x-lines); sweeps in flight per launch (t_fuse, 0 = as many as possible)
 * are capped so that a launch fits the array, which changes only the
 * schedule, never the result.  ST_EINVAL, before anything is enqueued, when
 * even one sweep does not fit (ceil(ny/8) * ceil(nz/8) above about 520,000
 * bundles, e.g. ny = nz = 6000), and for every argument stencil_gs rejects.
 * The caller owns u and f as for stencil_gs.
 */
int stencil_gs_noalloc(const st_grid *grid, int32_t dtype, void *u, const void *f,
                       const st_weights *w, int32_t bc, double bc_value, int32_t sweeps,
                       int32_t t_fuse, void *hip_stream);

/*
 * Bounded waits of the Gauss-Seidel wavefront.  A wave of the wavefront
 * kernel waits (spins) on its neighbours' progress counters.  Every such
 * wait is bounded: after `polls` polls (stencil_gs_spin_limit; default 2^24,
 * a few seconds), or once the device's abort word is raised, the wave gives
 * up, raises the abort word, and every wave of that and later launches on the
 * device then finishes its remaining work without waiting and exits: a
 * protocol fault ends the kernel instead of hanging the device.  The grid of
 * a launch that gave up holds partial results.
 *
 * stencil_sync        -- synchronizes hip_stream, then returns ST_EHIP if a
 *                        wavefront launch on the current device gave up since
 *                        the last stencil_sync (else ST_OK), and clears the
 *                        abort word and that status.  stencil_refine_solve
 *                        checks the same status after every round that used
 *                        the wavefront.
 * stencil_gs_abort    -- raises the abort word of `device` from the host (on a
 *                        stream of its own, so it lands while launches on
 *                        other streams run); returns once it is written.
 *                        ST_EINVAL for an unknown device.
 * stencil_gs_spin_limit -- polls of one wait before giving up, process-wide
 *                        (0 = default); ST_EINVAL outside 0..2^32-1.
 * The status and the abort word are per device, shared by every stream.
 */
int stencil_sync(void *hip_stream);
int stencil_gs_abort(int32_t device);
int stencil_gs_spin_limit(int64_t polls);

/*
 * stencil_rbgs -- `sweeps` red-black Gauss-Seidel sweeps: the alternative
 * ordering the paper names next to the lexicographic one (Sec. 3).  A sweep
 * updates, in place, every red site ((i + j + k) even, interior coordinates
 * counted from 0) and then every black site, with the same update and
 * operand order as stencil_gs; red sites read only old black values and
 * black sites the new red ones.  Run on the fused pass of stencil_jacobi:
 * one sweep is two time levels, so t_fuse (0 = automatic, else 1..4) sweeps
 * are applied per pass over memory and the pass alternates between u and
 * scratch.
 *  Arguments as for stencil_jacobi (u, scratch same size and dtype, not
 *  overlapping; result in u; stream-ordered).  Bit-identical to `sweeps`
 *  sequential red-black sweeps for every t_fuse.  ST_EINVAL for t_fuse
 *  outside 0..4 and the conditions listed for stencil_jacobi.
 */
int stencil_rbgs(const st_grid *grid, int32_t dtype, void *u, void *scratch, const void *f,
                 const st_weights *w, int32_t bc, double bc_value, int32_t sweeps,
                 int32_t t_fuse, void *hip_stream);

/*
 * stencil_residual -- FP64 residual of the h^2-scaled Poisson system
 * A u = f' with A u = 6c - s (the a = 0, b = 1/6 smoother's operator):
 *     r = f' - ((6*c) - s)
 * u: FP64 grid; fp: interior-only FP64 right-hand side (NULL = zero);
 * r_or_null: interior-only FP64 output or NULL; norm2_out (host pointer):
 * sum of r^2, reduced in a fixed tree order (deterministic run to run).
 * Synchronizes the stream before returning (*norm2_out is a host value).
 */
int stencil_residual(const st_grid *grid, const double *u, const double *fp, double *r_or_null,
                     double *norm2_out, void *hip_stream);

/*
 * stencil_refine_solve -- solve A u = f' (above) to ||r||/||f'|| <= rel_tol.
 *  inner_dtype ST_FP32 -- mixed-precision defect correction:
 *      loop: r = f' - A u (FP64 on the GPU); stop when rel <= rel_tol;
 *            e = inner_sweeps float sweeps of the method on A e = float(r)
 *                from e = 0 with zero ghosts and weights (0, 1/6, 1/6)
 *                (half the bytes per site of FP64);
 *            u = u + double(e) (FP64).
 *  inner_dtype ST_FP64 -- the plain FP64 method for comparison:
 *      loop: r = f' - A u; stop when rel <= rel_tol;
 *            u = inner_sweeps FP64 sweeps of the method on u itself with the
 *                right-hand side f' and weights (0, 1/6, 1/6).
 *  method      0 = Jacobi, 1 = Gauss-Seidel, 2 = red-black Gauss-Seidel
 *              (t_fuse then 0..4 sweeps per pass).
 *  u           FP64 grid: initial guess in, solution out; ghosts = Dirichlet.
 *  fp          interior-only FP64 right-hand side (h^2 f).
 *  t_fuse      fused sweeps per pass of the inner smoother (0 = automatic,
 *              else 1..8 or 16 as for stencil_jacobi).
 *  max_outer   residual checks followed by smoothing allowed; ST_ENOCONV if
 *              rel_tol is not reached after max_outer of them.
 *  outer_done, rel_res_out  (host pointers, may be NULL): smoothing rounds
 *              applied and the last relative residual.
 * Allocates its workspace internally and frees it before returning.
 * Synchronous.
 */
int stencil_refine_solve(const st_grid *grid, int32_t method, int32_t inner_dtype, double *u,
                         const double *fp, int32_t inner_sweeps, int32_t t_fuse, double rel_tol,
                         int32_t max_outer, int32_t *outer_done, double *rel_res_out,
                         void *hip_stream);

/*
 * stencil_mg_solve -- solve the h^2-scaled Poisson system A u = f' with
 * multigrid V-cycles whose smoother is one of this library's sweeps (the
 * paper names multigrid as the main user of these smoothers, Sec. 1), inside
 * the same FP64 defect correction as stencil_refine_solve:
 *     loop: r = f' - A u (FP64, deterministic norm); stop when
 *           ||r|| / ||f'|| <= rel_tol;  e = one V-cycle on A e = r in the
 *           inner precision (FP32: r rounded to float, every level in
 *           float);  u = u + e (FP64).
 *  Levels: the grid, then floor((n+1)/2) - 1 points per axis while every axis
 *  has >= 3 (512 -> 255 -> 127 -> ... -> 1).  Transfers: trilinear
 *  interpolation P between the level's points x_i = i/(n+1) and the coarse
 *  points X_I = I/(nc+1) (the nested full-weighting pair when n+1 is even);
 *  restriction = (h/H) P^T, i.e. the coarse right-hand side of the
 *  H^2-scaled coarse system.  V-cycle: e = 0, `pre` sweeps, restrict the
 *  residual, V-cycle one level down, e += P e_coarse, `post` sweeps; the
 *  coarsest level runs `coarse_sweeps` sweeps.
 *  smoother: 0 = weighted Jacobi, omega = 6/7 (weights a = b = g = 1/7, the
 *            fused Jacobi pass), 1 = lexicographic Gauss-Seidel (the
 *            wavefront), 2 = red-black Gauss-Seidel (the fused red-black pass);
 *            a = 0, b = g = 1/6 for 1 and 2.
 *  inner_dtype: ST_FP32 or ST_FP64.  u: FP64 padded grid (ghost width
 *  grid->halo, Dirichlet values in its ghosts are used by the FP64 residual;
 *  corrections have zero ghosts); fp: FP64 interior-only right-hand side.
 *  Synchronous.  *cycles_done = V-cycles applied, *rel_res_out = last
 *  relative residual (either may be NULL).  Returns ST_OK on convergence,
 *  ST_ENOCONV after max_cycles V-cycles; ST_EINVAL for smoother outside 0..2,
 *  pre/post outside 0..64, coarse_sweeps outside 1..4096, max_cycles < 0,
 *  rel_tol < 0 or NaN, NULL u/fp, and the grid conditions of stencil_jacobi;
 *  ST_EHIP on a device error or a Gauss-Seidel wavefront that gave up.  The
 *  library allocates one workspace (about 2.3x the grid in the inner
 *  precision) per call and frees it before returning.
 */
int stencil_mg_solve(const st_grid *grid, int32_t smoother, int32_t inner_dtype, double *u,
                     const double *fp, int32_t pre, int32_t post, int32_t coarse_sweeps,
                     double rel_tol, int32_t max_cycles, int32_t *cycles_done,
                     double *rel_res_out, void *hip_stream);

/* ------------------------------------------------------------------------
 * Continuous-batching job service.  Jobs (independent smoothing problems of
 * uneven sizes) are submitted from host memory at any time; a scheduler
 * thread admits them while the sum of their device footprints fits the HBM
 * budget and fewer than max_inflight are resident, uploads them into a
 * device pool, and runs every resident job's work inside shared persistent
 * kernels; jobs admitted while others run join the next batch launch, so
 * their work overlaps on the device.  A job's result does not depend on
 * which other jobs ran with it.
 */
typedef struct smooth_ctx smooth_ctx;

typedef struct {
    uint64_t hbm_budget_bytes;  /* device pool size; jobs must fit inside it */
    int32_t max_inflight;       /* resident jobs at most (>= 1) */
    int32_t device;             /* HIP device ordinal */
    int32_t t_fuse;             /* fused sweeps per Jacobi pass (0 = automatic, 1..8, 16) */
    int32_t sweeps_per_iteration; /* sweeps a resident job may do per batched iteration before
                                     the scheduler admits new jobs and finishes others: 0 = all
                                     of its sweeps (default); else at most this many (whole
                                     Jacobi passes, at least one).  Results do not depend on it. */
} smooth_config;

enum { SMOOTH_JACOBI = 0, SMOOTH_GS = 1 };
enum { SMOOTH_FP64 = 0, SMOOTH_FP32_REFINED = 1 };
enum { SMOOTH_QUEUED = 0, SMOOTH_RUNNING = 1, SMOOTH_DONE = 2, SMOOTH_FAILED = 3,
       SMOOTH_CANCELED = 4 };

/*
 * One smoothing job: `sweeps` sweeps of `method` on a grid of interior
 * extents nx, ny, nz with a ghost layer of width 1 (the st_grid limits apply:
 * one padded plane < 2^28 elements; Gauss-Seidel also needs ny, nz <= 8192).
 *  precision SMOOTH_FP64: plain FP64 sweeps (bit-identical to stencil_jacobi
 *            / stencil_gs).  SMOOTH_FP32_REFINED: one defect-correction step,
 *            r = (one FP64 update of u0) - u0, `sweeps` float sweeps of
 *            e <- (center*e) + (neighbor*s_e) + r from e = 0 with zero ghosts,
 *            u = u0 + e in FP64 (equal to the plain result in exact
 *            arithmetic; within float rounding of the correction in practice).
 *  input_host  (nz+2)(ny+2)(nx+2) doubles, read during the call to
 *              smooth_submit's admission (keep valid until DONE/FAILED/CANCELED).
 *  output_host same size, written before the job turns DONE.
 */
typedef struct {
    int64_t nx, ny, nz;
    int32_t method;
    int32_t precision;
    int32_t sweeps;
    int32_t reserved;
    st_weights weights;
    const double *input_host;
    double *output_host;
} smooth_job;

/* Per-job timestamps (steady clock, ns) and accounting.  A job's latency
 * t_done - t_submit splits into queue (t_admit - t_submit: waiting for pool
 * space or a slot), upload (t_uploaded - t_admit: host-to-device copy of the
 * input, including the wait for a copy thread), compute (t_computed -
 * t_uploaded: the batched iterations that ran its sweeps, including the wait
 * for the next iteration; t_start marks its first launch) and download
 * (t_done - t_computed: device-to-host copy of the result). */
typedef struct {
    int64_t t_submit_ns, t_admit_ns, t_start_ns, t_done_ns;
    uint64_t footprint_bytes;   /* device bytes the job held while resident */
    double lups;                /* lattice-site updates performed (interior sites * sweeps) */
    int32_t batch_id;           /* launch batch that ran the job's sweeps */
    int32_t reserved;
    int64_t t_uploaded_ns;      /* input resident on the device */
    int64_t t_computed_ns;      /* last iteration of the job completed */
} smooth_stats;

/* Create a service: allocates the device pool (hbm_budget_bytes) and starts
 * the scheduler thread.  ST_ENOMEM if the pool cannot be allocated. */
int smooth_init(const smooth_config *cfg, smooth_ctx **out);

/* Queue a job (non-blocking).  ST_EINVAL for bad extents/method/precision/
 * sweeps or a footprint larger than the whole budget; *job_id receives an id
 * unique within the context. */
int smooth_submit(smooth_ctx *ctx, const smooth_job *job, uint64_t *job_id);

/* Non-blocking state query; stats may be NULL.  ST_ENOENT for unknown ids. */
int smooth_poll(smooth_ctx *ctx, uint64_t job_id, int32_t *state, smooth_stats *stats);

/* Block until every submitted job is DONE, FAILED or CANCELED (timeout_ms < 0
 * waits forever).  ST_EBUSY on timeout. */
int smooth_wait_all(smooth_ctx *ctx, int64_t timeout_ms);

/* Service-wide counters: pool high-water mark, batches launched, jobs done. */
typedef struct {
    uint64_t pool_bytes, footprint_high_water, footprint_now;
    int64_t batches, jobs_done, jobs_failed, jobs_canceled;
    int32_t max_resident_seen, reserved;
} smooth_service_stats;
int smooth_service_info(smooth_ctx *ctx, smooth_service_stats *out);

/* Cancel queued jobs (CANCELED), let resident jobs finish, stop the thread,
 * free the pool and the context. */
int smooth_shutdown(smooth_ctx *ctx);

/* Human-readable name of a status code, and the calling thread's last error. */
const char *stencil_strerror(int status);
const char *stencil_last_error(void);

/* Library version string. */
const char *stencil_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_H */
