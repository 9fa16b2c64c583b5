// api.cpp -- the C ABI of libstencil (include/stencil.h): argument checks,
// the pass schedules, and the refinement loop.  All numerical work is done by
// the HIP kernels of jacobi_impl.h (one unit per depth, jacobi_t<N>.hip),
// gs.hip and aux.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "../../include/stencil.h"
#include "internal.h"

namespace stk {

static thread_local std::string t_last_error;

void set_error(const std::string &msg) { t_last_error = msg; }

}  // namespace stk

using namespace stk;

namespace {

int fail(int status, const std::string &msg) {
    set_error(msg);
    return status;
}

int hip_fail(hipError_t e, const char *where) {
    return fail(ST_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, where)                      \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

int check_grid(const st_grid *g, Geom *out) {
    if (!g) return fail(ST_EINVAL, "grid is NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1)
        return fail(ST_EINVAL, "interior extents must be >= 1");
    if (g->halo < 1) return fail(ST_EINVAL, "halo must be >= 1");
    const int64_t px = g->nx + 2 * (int64_t)g->halo, py = g->ny + 2 * (int64_t)g->halo,
                  pz = g->nz + 2 * (int64_t)g->halo;
    // kernels address a plane with 32-bit byte offsets (8-byte elements)
    if (px * py >= (int64_t)1 << 28 || pz >= (int64_t)1 << 31 || g->halo > 4096)
        return fail(ST_EINVAL, "grid too large (one padded plane must hold < 2^28 elements)");
    out->nx = (int)g->nx;
    out->ny = (int)g->ny;
    out->nz = (int)g->nz;
    out->h = g->halo;
    out->px = px;
    out->py = py;
    out->pz = pz;
    return ST_OK;
}

bool valid_t(int t) { return (t >= 0 && t <= 8) || t == 16; }

// Automatic depth, measured at 512^3 on MI355X (100 sweeps; 32 with f):
// FP64 t=5 (559 us per pass, 112 us per sweep; t=4 481 us, 120 per sweep;
// t=6 660 us, 110 per sweep, but 100 is not a multiple of 6), with f t=4
// (32 sweeps in 8 passes; t=5 needs 8 passes too, two of them of one
// sweep); FP32 t=5, with f t=6.
int auto_t(int dtype, bool rhs) {
    if (dtype == ST_FP32) return rhs ? 6 : 5;
    return rhs ? 4 : 5;
}

// Pass schedule: floor(S/t) passes of t plus one pass of the remainder (every
// depth 1..8 is compiled); if the count is odd the smallest pass with >= 2
// sweeps is split in two so the result lands in u, else a final copy is
// needed.  any_parity: keep an odd count (the caller swaps its grids).
std::vector<int> jacobi_plan(int dtype, bool rhs, int sweeps, int t_fuse, bool *final_copy,
                             bool any_parity = false) {
    int t = t_fuse == 0 ? auto_t(dtype, rhs) : t_fuse;
    if (t > 8) t = 8;  // at most 8 levels fit on chip per pass
    std::vector<int> p;
    for (int i = 0; i < sweeps / t; ++i) p.push_back(t);
    if (sweeps % t) p.push_back(sweeps % t);
    *final_copy = false;
    if (p.size() % 2 == 1 && !any_parity) {
        int best = -1;
        for (size_t i = 0; i < p.size(); ++i)
            if (p[i] >= 2 && (best < 0 || p[i] < p[best])) best = (int)i;
        if (best >= 0) {
            const int lo = p[best] / 2;
            const int hi = p[best] - lo;
            p[best] = hi;
            p.insert(p.begin() + best + 1, lo);
        } else {
            *final_copy = true;
        }
    }
    return p;
}

bool overlaps(const void *a, const void *b, size_t bytes) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + bytes && y < x + bytes;
}

// Red-black sweeps per pass (defined below).
int rb_sweeps_per_pass(int t_fuse, bool fp32, bool rhs);

// The fused passes of `sweeps` Jacobi (rb = false) or red-black (rb = true)
// sweeps, alternating between *u and *scratch.  The result is returned in *u.
// owned: the caller owns both grids and their ghost cells are equal, so an
// odd number of passes leaves the result in the other grid and the two
// pointers are swapped; otherwise the schedule has an even count (a pass is
// split) or ends with a copy of the interior back to *u.
int run_fused(bool rb, const Geom &g, bool fp32, void **u, void **scratch, bool owned,
              const void *f, double a, double b, double gw, int sweeps, int t_fuse,
              hipStream_t s) {
    if (sweeps == 0) return ST_OK;
    bool fc = false;
    const int t = rb ? rb_sweeps_per_pass(t_fuse, fp32, f != nullptr) : t_fuse;
    std::vector<int> plan =
        jacobi_plan(fp32 ? ST_FP32 : ST_FP64, f != nullptr, sweeps, t, &fc, owned);
    HIP_TRY(launch_copy_ghosts(fp32, g, *u, *scratch, s), "ghost copy");
    const void *src = *u;
    void *dst = *scratch;
    for (int n : plan) {
        if (rb)
            HIP_TRY(launch_rbgs_pass(fp32, n, g, src, dst, f, a, b, gw, s), "red-black pass");
        else
            HIP_TRY(launch_jacobi_pass(fp32, n, g, src, dst, f, a, b, gw, 0, s), "jacobi pass");
        void *tmp = const_cast<void *>(src);
        src = dst;
        dst = tmp;
    }
    if (fc) HIP_TRY(launch_copy_interior(fp32, g, *scratch, *u, s), "final copy");
    if (owned && plan.size() % 2 == 1) std::swap(*u, *scratch);
    return ST_OK;
}

int run_jacobi(const Geom &g, bool fp32, void *u, void *scratch, const void *f, double a,
               double b, double gw, int sweeps, int t_fuse, hipStream_t s) {
    return run_fused(false, g, fp32, &u, &scratch, false, f, a, b, gw, sweeps, t_fuse, s);
}

// Red-black sweeps per pass: at most 4 (8 levels on chip).  Automatic: FP64
// 2 with a right-hand side and 3 without, FP32 3.  512^3 on MI355X, 32 sweeps
// with a right-hand side (the inner solve of the refinement) at 1/2/3/4
// sweeps per pass: FP64 23.3/14.4/23.2/35.8 ms, FP32 17.6/11.6/8.1/9.9 ms;
// without one, 100 sweeps: FP64 50.2/25.2/24.9/30.2 ms, FP32 3 per pass the
// fastest.
int rb_sweeps_per_pass(int t_fuse, bool fp32, bool rhs) {
    int t = t_fuse == 0 ? (fp32 || !rhs ? 3 : 2) : t_fuse;
    return t > 4 ? 4 : t;
}

// the same schedule rule as Jacobi, counted in red-black sweeps
int run_rbgs(const Geom &g, bool fp32, void *u, void *scratch, const void *f, double a, double b,
             double gw, int sweeps, int t_fuse, hipStream_t s) {
    return run_fused(true, g, fp32, &u, &scratch, false, f, a, b, gw, sweeps, t_fuse, s);
}

// Sweeps in flight per wavefront launch: t_fuse, or all (at most 4095).
int run_gs(const Geom &g, bool fp32, void *u, const void *f, double a, double b, double gw,
           int sweeps, int t_fuse, hipStream_t s) {
    int per = t_fuse == 0 ? 4095 : t_fuse;
    if (per > 4095) per = 4095;
    // one launch holds fewer than 2^31 (sweep, bundle) items
    const int64_t bundles = (int64_t)((g.ny + 7) / 8) * ((g.nz + 7) / 8);
    if ((int64_t)per * bundles >= ((int64_t)1 << 31)) per = (int)((((int64_t)1 << 31) - 1) / bundles);
    for (int done = 0; done < sweeps; done += per) {
        const int n = sweeps - done < per ? sweeps - done : per;
        HIP_TRY(launch_gs(fp32, g, u, f, a, b, gw, n, s), "gauss-seidel launch");
    }
    return ST_OK;
}

// The same launches with the workspace in the library's static device array:
// sweeps per launch are capped so that one launch's workspace fits it.
int run_gs_noalloc(const Geom &g, bool fp32, void *u, const void *f, double a, double b,
                   double gw, int sweeps, int t_fuse, hipStream_t s) {
    int per = t_fuse == 0 ? 4095 : t_fuse;
    if (per > 4095) per = 4095;
    while (per > 1 && gs_workspace_bytes(per, g.ny, g.nz) > GS_NOALLOC_BYTES) --per;
    for (int done = 0; done < sweeps; done += per) {
        const int n = sweeps - done < per ? sweeps - done : per;
        HIP_TRY(launch_gs_noalloc(fp32, g, u, f, a, b, gw, n, s), "gauss-seidel launch");
    }
    return ST_OK;
}

// ST_EHIP (and clears the flag) if a wavefront launch on the current device
// gave up waiting; synchronizes s.
int check_gs_status(hipStream_t s) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "device");
    uint32_t st = 0;
    HIP_TRY(gs_status(dev, s, true, &st), "gauss-seidel status");
    if (st & 1u)
        return fail(ST_EHIP, "a Gauss-Seidel wavefront launch gave up waiting (spin limit "
                             "reached or abort requested); its grid holds partial results");
    return ST_OK;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return hipMalloc(&p, bytes ? bytes : 1); }
};

}  // namespace

namespace stk {
std::vector<int> jacobi_pass_plan(bool fp32, bool rhs, int sweeps, int t_fuse, bool *final_copy) {
    return jacobi_plan(fp32 ? ST_FP32 : ST_FP64, rhs, sweeps, t_fuse, final_copy);
}
}  // namespace stk

extern "C" {

const char *stencil_version(void) { return "libstencil 0.1 (gfx950)"; }

const char *stencil_strerror(int status) {
    switch (status) {
        case ST_OK: return "ok";
        case ST_EINVAL: return "invalid argument";
        case ST_ENOMEM: return "out of memory";
        case ST_EHIP: return "HIP runtime error";
        case ST_EBUSY: return "busy";
        case ST_ENOENT: return "no such job";
        case ST_ENOCONV: return "not converged";
        case ST_ECANCELED: return "canceled";
        default: return "unknown status";
    }
}

const char *stencil_last_error(void) { return t_last_error.c_str(); }

int stencil_jacobi_plan(int32_t dtype, int32_t has_rhs, int32_t sweeps, int32_t t_fuse, int32_t *passes,
                        int32_t *t_list, int32_t max_list, int32_t *final_copy) {
    if (dtype != ST_FP64 && dtype != ST_FP32) return fail(ST_EINVAL, "dtype must be FP64 or FP32");
    if (sweeps < 0) return fail(ST_EINVAL, "sweeps must be >= 0");
    if (!valid_t(t_fuse)) return fail(ST_EINVAL, "t_fuse must be 0..8 or 16");
    if (!passes) return fail(ST_EINVAL, "passes is NULL");
    bool fc = false;
    std::vector<int> p =
        sweeps ? jacobi_plan(dtype, has_rhs != 0, sweeps, t_fuse, &fc) : std::vector<int>();
    *passes = (int32_t)p.size();
    if (t_list)
        for (int i = 0; i < (int)p.size() && i < max_list; ++i) t_list[i] = p[i];
    if (final_copy) *final_copy = fc ? 1 : 0;
    return ST_OK;
}

int stencil_jacobi_tiles(const st_grid *grid, int32_t dtype, int32_t has_rhs, int32_t levels,
                         int32_t *tile_w, int32_t *tile_h, int32_t *tiles, int32_t *interior) {
    Geom g;
    int rc = check_grid(grid, &g);
    if (rc) return rc;
    if (dtype != ST_FP64 && dtype != ST_FP32) return fail(ST_EINVAL, "dtype must be FP64 or FP32");
    if (levels < 1 || levels > 8) return fail(ST_EINVAL, "levels must be 1..8");
    const bool fp32 = dtype == ST_FP32;
    const JacTileCfg c = jacobi_tile_cfg(fp32, levels, has_rhs != 0);
    int nt = 0, ni = 0;
    jacobi_tile_count(fp32, levels, has_rhs != 0, g, &nt, &ni);
    if (tile_w) *tile_w = c.ow();
    if (tile_h) *tile_h = c.oh();
    if (tiles) *tiles = nt;
    if (interior) *interior = ni;
    return ST_OK;
}

int stencil_jacobi(const st_grid *grid, int32_t dtype, void *u, void *scratch, const void *f,
                   const st_weights *w, int32_t bc, double bc_value, int32_t sweeps,
                   int32_t t_fuse, void *hip_stream) {
    Geom g;
    int rc = check_grid(grid, &g);
    if (rc) return rc;
    if (dtype != ST_FP64 && dtype != ST_FP32) return fail(ST_EINVAL, "dtype must be FP64 or FP32");
    if (!u || !scratch) return fail(ST_EINVAL, "u and scratch must be device pointers");
    if (!w) return fail(ST_EINVAL, "weights is NULL");
    if (bc != ST_BC_KEEP && bc != ST_BC_CONST) return fail(ST_EINVAL, "bc must be KEEP or CONST");
    if (sweeps < 0) return fail(ST_EINVAL, "sweeps must be >= 0");
    if (!valid_t(t_fuse)) return fail(ST_EINVAL, "t_fuse must be 0..8 or 16");
    const bool fp32 = dtype == ST_FP32;
    const size_t bytes = (size_t)g.count() * (fp32 ? 4 : 8);
    if (overlaps(u, scratch, bytes)) return fail(ST_EINVAL, "u and scratch overlap");
    if (!std::isfinite(w->center) || !std::isfinite(w->neighbor) || !std::isfinite(w->rhs))
        return fail(ST_EINVAL, "weights must be finite");
    hipStream_t s = (hipStream_t)hip_stream;
    if (bc == ST_BC_CONST) HIP_TRY(launch_fill_ghosts(fp32, g, u, bc_value, s), "ghost fill");
    return run_jacobi(g, fp32, u, scratch, f, w->center, w->neighbor, f ? w->rhs : 0.0, sweeps,
                      t_fuse, s);
}

int stencil_rbgs(const st_grid *grid, int32_t dtype, void *u, void *scratch, const void *f,
                 const st_weights *w, int32_t bc, double bc_value, int32_t sweeps,
                 int32_t t_fuse, void *hip_stream) {
    Geom g;
    int rc = check_grid(grid, &g);
    if (rc) return rc;
    if (dtype != ST_FP64 && dtype != ST_FP32) return fail(ST_EINVAL, "dtype must be FP64 or FP32");
    if (!u || !scratch) return fail(ST_EINVAL, "u and scratch must be device pointers");
    if (!w) return fail(ST_EINVAL, "weights is NULL");
    if (bc != ST_BC_KEEP && bc != ST_BC_CONST) return fail(ST_EINVAL, "bc must be KEEP or CONST");
    if (sweeps < 0) return fail(ST_EINVAL, "sweeps must be >= 0");
    if (t_fuse < 0 || t_fuse > 4) return fail(ST_EINVAL, "t_fuse must be 0..4 for red-black");
    const bool fp32 = dtype == ST_FP32;
    const size_t bytes = (size_t)g.count() * (fp32 ? 4 : 8);
    if (overlaps(u, scratch, bytes)) return fail(ST_EINVAL, "u and scratch overlap");
    if (!std::isfinite(w->center) || !std::isfinite(w->neighbor) || !std::isfinite(w->rhs))
        return fail(ST_EINVAL, "weights must be finite");
    hipStream_t s = (hipStream_t)hip_stream;
    if (bc == ST_BC_CONST) HIP_TRY(launch_fill_ghosts(fp32, g, u, bc_value, s), "ghost fill");
    return run_rbgs(g, fp32, u, scratch, f, w->center, w->neighbor, f ? w->rhs : 0.0, sweeps,
                    t_fuse, s);
}

int stencil_gs(const st_grid *grid, int32_t dtype, void *u, const void *f, const st_weights *w,
               int32_t bc, double bc_value, int32_t sweeps, int32_t t_fuse, void *hip_stream) {
    Geom g;
    int rc = check_grid(grid, &g);
    if (rc) return rc;
    if (dtype != ST_FP64 && dtype != ST_FP32) return fail(ST_EINVAL, "dtype must be FP64 or FP32");
    if (!u) return fail(ST_EINVAL, "u must be a device pointer");
    if (!w) return fail(ST_EINVAL, "weights is NULL");
    if (bc != ST_BC_KEEP && bc != ST_BC_CONST) return fail(ST_EINVAL, "bc must be KEEP or CONST");
    if (sweeps < 0) return fail(ST_EINVAL, "sweeps must be >= 0");
    if (!valid_t(t_fuse)) return fail(ST_EINVAL, "t_fuse must be 0..8 or 16");
    if (g.ny > 8192 || g.nz > 8192)
        return fail(ST_EINVAL, "Gauss-Seidel supports ny, nz <= 8192");
    if (!std::isfinite(w->center) || !std::isfinite(w->neighbor) || !std::isfinite(w->rhs))
        return fail(ST_EINVAL, "weights must be finite");
    const bool fp32 = dtype == ST_FP32;
    hipStream_t s = (hipStream_t)hip_stream;
    if (bc == ST_BC_CONST) HIP_TRY(launch_fill_ghosts(fp32, g, u, bc_value, s), "ghost fill");
    if (sweeps == 0) return ST_OK;
    return run_gs(g, fp32, u, f, w->center, w->neighbor, f ? w->rhs : 0.0, sweeps, t_fuse, s);
}

int stencil_gs_noalloc(const st_grid *grid, int32_t dtype, void *u, const void *f,
                       const st_weights *w, int32_t bc, double bc_value, int32_t sweeps,
                       int32_t t_fuse, void *hip_stream) {
    Geom g;
    int rc = check_grid(grid, &g);
    if (rc) return rc;
    if (dtype != ST_FP64 && dtype != ST_FP32) return fail(ST_EINVAL, "dtype must be FP64 or FP32");
    if (!u) return fail(ST_EINVAL, "u must be a device pointer");
    if (!w) return fail(ST_EINVAL, "weights is NULL");
    if (bc != ST_BC_KEEP && bc != ST_BC_CONST) return fail(ST_EINVAL, "bc must be KEEP or CONST");
    if (sweeps < 0) return fail(ST_EINVAL, "sweeps must be >= 0");
    if (!valid_t(t_fuse)) return fail(ST_EINVAL, "t_fuse must be 0..8 or 16");
    if (g.ny > 8192 || g.nz > 8192)
        return fail(ST_EINVAL, "Gauss-Seidel supports ny, nz <= 8192");
    if (gs_workspace_bytes(1, g.ny, g.nz) > GS_NOALLOC_BYTES)
        return fail(ST_EINVAL, "grid too large for stencil_gs_noalloc: the workspace of one "
                               "sweep (8 bytes per 8x8 bundle of x-lines) exceeds its 4 MiB "
                               "static device array; use stencil_gs");
    if (!std::isfinite(w->center) || !std::isfinite(w->neighbor) || !std::isfinite(w->rhs))
        return fail(ST_EINVAL, "weights must be finite");
    const bool fp32 = dtype == ST_FP32;
    hipStream_t s = (hipStream_t)hip_stream;
    if (bc == ST_BC_CONST) HIP_TRY(launch_fill_ghosts(fp32, g, u, bc_value, s), "ghost fill");
    if (sweeps == 0) return ST_OK;
    return run_gs_noalloc(g, fp32, u, f, w->center, w->neighbor, f ? w->rhs : 0.0, sweeps,
                          t_fuse, s);
}

int stencil_sync(void *hip_stream) { return check_gs_status((hipStream_t)hip_stream); }

int stencil_gs_abort(int32_t device) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
        return fail(ST_EINVAL, "no such HIP device");
    HIP_TRY(gs_abort(device), "gauss-seidel abort");
    return ST_OK;
}

int stencil_gs_spin_limit(int64_t polls) {
    if (polls < 0 || polls > 0xffffffffll) return fail(ST_EINVAL, "polls must be 0..2^32-1");
    gs_set_spin_limit((uint32_t)polls);
    return ST_OK;
}

int stencil_residual(const st_grid *grid, const double *u, const double *fp, double *r_or_null,
                     double *norm2_out, void *hip_stream) {
    Geom g;
    int rc = check_grid(grid, &g);
    if (rc) return rc;
    if (!u) return fail(ST_EINVAL, "u must be a device pointer");
    if (!norm2_out) return fail(ST_EINVAL, "norm2_out is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    const int nb = residual_partial_count(g);
    DevBuf part;
    HIP_TRY(part.alloc(((size_t)nb + 1) * sizeof(double)), "residual workspace");
    double *partials = (double *)part.p;
    HIP_TRY(launch_residual_poisson(g, u, fp, r_or_null, nullptr, partials, nullptr, s),
            "residual");
    HIP_TRY(launch_sum_partials(partials, nb, partials + nb, s), "residual sum");
    double host = 0.0;
    HIP_TRY(hipMemcpyAsync(&host, partials + nb, sizeof(double), hipMemcpyDeviceToHost, s),
            "residual copy");
    HIP_TRY(hipStreamSynchronize(s), "residual sync");
    *norm2_out = host;
    return ST_OK;
}

int stencil_refine_solve(const st_grid *grid, int32_t method, int32_t inner_dtype, double *u,
                         const double *fp, int32_t inner_sweeps, int32_t t_fuse, double rel_tol,
                         int32_t max_outer, int32_t *outer_done, double *rel_res_out,
                         void *hip_stream) {
    Geom g;
    int rc = check_grid(grid, &g);
    if (rc) return rc;
    if (method < 0 || method > 2)
        return fail(ST_EINVAL, "method must be 0 (Jacobi), 1 (GS) or 2 (red-black GS)");
    if (inner_dtype != ST_FP64 && inner_dtype != ST_FP32)
        return fail(ST_EINVAL, "inner_dtype must be FP64 or FP32");
    if (!u || !fp) return fail(ST_EINVAL, "u and fp must be device pointers");
    if (inner_sweeps < 1) return fail(ST_EINVAL, "inner_sweeps must be >= 1");
    if (max_outer < 0) return fail(ST_EINVAL, "max_outer must be >= 0");
    if (!valid_t(t_fuse)) return fail(ST_EINVAL, "t_fuse must be 0..8 or 16");
    if (method == 2 && t_fuse > 4) return fail(ST_EINVAL, "t_fuse must be 0..4 for red-black");
    if (!(rel_tol >= 0.0)) return fail(ST_EINVAL, "rel_tol must be >= 0");
    if (method == 1 && (g.ny > 8192 || g.nz > 8192))
        return fail(ST_EINVAL, "Gauss-Seidel supports ny, nz <= 8192");
    hipStream_t s = (hipStream_t)hip_stream;
    const bool f32 = inner_dtype == ST_FP32;
    const int64_t ni = g.interior(), np = g.count();
    const int nb = residual_partial_count(g);

    DevBuf part, rbuf, ebuf, sbuf;
    HIP_TRY(part.alloc(((size_t)nb + 2) * sizeof(double)), "refine workspace");
    double *partials = (double *)part.p;
    double *dsum = partials + nb;
    if (f32) {
        HIP_TRY(rbuf.alloc((size_t)ni * sizeof(float)), "refine workspace");
        HIP_TRY(ebuf.alloc((size_t)np * sizeof(float)), "refine workspace");
        if (method != 1) HIP_TRY(sbuf.alloc((size_t)np * sizeof(float)), "refine workspace");
    } else if (method != 1) {
        HIP_TRY(sbuf.alloc((size_t)np * sizeof(double)), "refine workspace");
    }
    // ||f'|| with the same deterministic reduction (the residual of u = 0 is f')
    HIP_TRY(launch_residual_poisson(g, nullptr, fp, nullptr, nullptr, partials, nullptr, s),
            "norm f");
    HIP_TRY(launch_sum_partials(partials, nb, dsum + 1, s), "norm f");
    double ff = 0.0;
    HIP_TRY(hipMemcpyAsync(&ff, dsum + 1, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    const double nf = std::sqrt(ff);
    if (f32) {
        HIP_TRY(hipMemsetAsync(ebuf.p, 0, (size_t)np * sizeof(float), s), "memset");
        if (sbuf.p) HIP_TRY(hipMemsetAsync(sbuf.p, 0, (size_t)np * sizeof(float), s), "memset");
    }
    const st_weights pw = {0.0, 1.0 / 6.0, 1.0 / 6.0};
    // the FP32 correction and its scratch grid (both owned here: an odd pass
    // count swaps them instead of splitting a pass)
    void *e = ebuf.p, *es = sbuf.p;
    int outer = 0;
    double rel = INFINITY;
    int status = ST_ENOCONV;
    for (;;) {
        HIP_TRY(launch_residual_poisson(g, u, fp, nullptr, f32 ? (float *)rbuf.p : nullptr,
                                        partials, nullptr, s), "residual");
        HIP_TRY(launch_sum_partials(partials, nb, dsum, s), "residual sum");
        double rr = 0.0;
        HIP_TRY(hipMemcpyAsync(&rr, dsum, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        rel = nf > 0.0 ? std::sqrt(rr) / nf : std::sqrt(rr);
        if (rel <= rel_tol) {
            status = ST_OK;
            break;
        }
        if (outer >= max_outer) break;
        if (f32) {
            // e = 0 (ghosts stay 0), then inner_sweeps float sweeps on A e = r
            HIP_TRY(hipMemsetAsync(e, 0, (size_t)np * sizeof(float), s), "memset");
            if (method == 1)
                rc = run_gs(g, true, e, rbuf.p, pw.center, pw.neighbor, pw.rhs, inner_sweeps,
                            t_fuse, s);
            else
                rc = run_fused(method == 2, g, true, &e, &es, true, rbuf.p, pw.center,
                               pw.neighbor, pw.rhs, inner_sweeps, t_fuse, s);
            if (rc) return rc;
            HIP_TRY(launch_correct(g, u, e, true, s), "correct");
        } else {
            // the plain FP64 method: smooth u itself with the right-hand side
            if (method == 0)
                rc = run_jacobi(g, false, u, sbuf.p, fp, pw.center, pw.neighbor, pw.rhs,
                                inner_sweeps, t_fuse, s);
            else if (method == 2)
                rc = run_rbgs(g, false, u, sbuf.p, fp, pw.center, pw.neighbor, pw.rhs,
                              inner_sweeps, t_fuse, s);
            else
                rc = run_gs(g, false, u, fp, pw.center, pw.neighbor, pw.rhs, inner_sweeps,
                            t_fuse, s);
            if (rc) return rc;
        }
        ++outer;
        if (method == 1) {  // the round's wavefront launches must have completed normally
            rc = check_gs_status(s);
            if (rc) return rc;
        }
    }
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (outer_done) *outer_done = outer;
    if (rel_res_out) *rel_res_out = rel;
    if (status == ST_ENOCONV) set_error("relative residual above rel_tol after max_outer steps");
    return status;
}

int stencil_mg_solve(const st_grid *grid, int32_t smoother, int32_t inner_dtype, double *u,
                     const double *fp, int32_t pre, int32_t post, int32_t coarse_sweeps,
                     double rel_tol, int32_t max_cycles, int32_t *cycles_done,
                     double *rel_res_out, void *hip_stream) {
    Geom g;
    int rc = check_grid(grid, &g);
    if (rc) return rc;
    if (smoother < 0 || smoother > 2)
        return fail(ST_EINVAL, "smoother must be 0 (weighted Jacobi), 1 (GS) or 2 (red-black GS)");
    if (inner_dtype != ST_FP64 && inner_dtype != ST_FP32)
        return fail(ST_EINVAL, "inner_dtype must be FP64 or FP32");
    if (!u || !fp) return fail(ST_EINVAL, "u and fp must be device pointers");
    if (pre < 0 || post < 0 || pre > 64 || post > 64)
        return fail(ST_EINVAL, "pre and post must be 0..64");
    if (coarse_sweeps < 1 || coarse_sweeps > 4096)
        return fail(ST_EINVAL, "coarse_sweeps must be 1..4096");
    if (max_cycles < 0) return fail(ST_EINVAL, "max_cycles must be >= 0");
    if (!(rel_tol >= 0.0)) return fail(ST_EINVAL, "rel_tol must be >= 0");
    if (smoother == 1 && (g.ny > 8192 || g.nz > 8192))
        return fail(ST_EINVAL, "Gauss-Seidel supports ny, nz <= 8192");
    hipStream_t s = (hipStream_t)hip_stream;
    const bool f32 = inner_dtype == ST_FP32;
    const size_t es = f32 ? sizeof(float) : sizeof(double);

    // levels: the grid itself, then floor((n+1)/2) - 1 points per axis while
    // every axis has >= 3
    std::vector<Geom> lv(1, g);
    while (lv.back().nx >= 3 && lv.back().ny >= 3 && lv.back().nz >= 3 && lv.size() < 32) {
        Geom c;
        c.nx = mg_coarse_n(lv.back().nx);
        c.ny = mg_coarse_n(lv.back().ny);
        c.nz = mg_coarse_n(lv.back().nz);
        c.h = 1;
        c.px = c.nx + 2;
        c.py = c.ny + 2;
        c.pz = c.nz + 2;
        lv.push_back(c);
    }
    const int nlev = (int)lv.size();
    // one device allocation: per level e, its Jacobi/red-black scratch, r and
    // res, then the transfer tables
    auto up = [](size_t n) { return (n + 255) / 256 * 256; };
    struct Off { size_t e, es, r, res; };
    std::vector<Off> off(nlev);
    size_t total = 0;
    for (int l = 0; l < nlev; ++l) {
        off[l].e = total;
        total += up((size_t)lv[l].count() * es);
        off[l].es = total;
        if (smoother != 1) total += up((size_t)lv[l].count() * es);
        off[l].r = total;
        total += up((size_t)lv[l].interior() * es);
        off[l].res = total;
        total += up((size_t)lv[l].interior() * es);
    }
    std::vector<unsigned char> tb;
    std::vector<MgTables> tabs(nlev > 1 ? nlev - 1 : 0);
    for (int l = 0; l + 1 < nlev; ++l)
        if (!mg_build_tables(f32, lv[l], tb, tabs[l]))
            return fail(ST_EINVAL, "multigrid transfer support too wide for this grid");
    const size_t tab_off = total;
    total += up(tb.size());
    // partial sums of the restriction (one level at a time: the largest)
    size_t rtmp = 0;
    for (int l = 0; l + 1 < nlev; ++l)
        rtmp = std::max(rtmp, mg_restrict_tmp_bytes(f32, lv[l], lv[l + 1]));
    const size_t rtmp_off = total;
    total += up(rtmp);
    const int nb = residual_partial_count(g);
    const size_t part_off = total;
    total += up(((size_t)nb + 2) * sizeof(double));
    DevBuf work;
    HIP_TRY(work.alloc(total), "multigrid workspace");
    unsigned char *base = (unsigned char *)work.p;
    if (!tb.empty())
        HIP_TRY(hipMemcpyAsync(base + tab_off, tb.data(), tb.size(), hipMemcpyHostToDevice, s),
                "multigrid tables");
    for (auto &t : tabs) t.dev = base + tab_off;
    auto E = [&](int l) { return (void *)(base + off[l].e); };
    auto ES = [&](int l) { return (void *)(base + off[l].es); };
    auto R = [&](int l) { return (void *)(base + off[l].r); };
    auto RES = [&](int l) { return (void *)(base + off[l].res); };
    double *partials = (double *)(base + part_off);
    double *dsum = partials + nb;

    // the correction of each level and its scratch grid: an odd number of
    // smoothing passes swaps the two instead of splitting a pass
    std::vector<void *> e(nlev), esc(nlev);
    for (int l = 0; l < nlev; ++l) e[l] = E(l), esc[l] = ES(l);
    auto smooth = [&](int l, int sweeps) -> int {
        if (sweeps <= 0) return ST_OK;
        if (smoother == 0)  // weighted Jacobi, omega = 6/7
            return run_fused(false, lv[l], f32, &e[l], &esc[l], true, R(l), 1.0 / 7.0, 1.0 / 7.0,
                             1.0 / 7.0, sweeps, 0, s);
        if (smoother == 2)
            return run_fused(true, lv[l], f32, &e[l], &esc[l], true, R(l), 0.0, 1.0 / 6.0,
                             1.0 / 6.0, sweeps, 0, s);
        return run_gs(lv[l], f32, e[l], R(l), 0.0, 1.0 / 6.0, 1.0 / 6.0, sweeps, 0, s);
    };
    auto zero = [&](int l) {
        return hipMemsetAsync(e[l], 0, (size_t)lv[l].count() * es, s);
    };
    if (smoother != 1)  // scratch ghosts start at 0 (run_jacobi / run_rbgs copy them anyway)
        for (int l = 0; l < nlev; ++l)
            HIP_TRY(hipMemsetAsync(ES(l), 0, (size_t)lv[l].count() * es, s), "memset");

    // ||f'|| with the same deterministic reduction as the residual
    HIP_TRY(launch_residual_poisson(g, nullptr, fp, nullptr, nullptr, partials, nullptr, s),
            "norm f");
    HIP_TRY(launch_sum_partials(partials, nb, dsum + 1, s), "norm f");
    double ff = 0.0;
    HIP_TRY(hipMemcpyAsync(&ff, dsum + 1, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
    HIP_TRY(hipStreamSynchronize(s), "sync");
    const double nf = std::sqrt(ff);

    int cyc = 0, status = ST_ENOCONV;
    double rel = INFINITY;
    for (;;) {
        HIP_TRY(launch_residual_poisson(g, u, fp, f32 ? nullptr : (double *)R(0),
                                        f32 ? (float *)R(0) : nullptr, partials, nullptr, s),
                "residual");
        HIP_TRY(launch_sum_partials(partials, nb, dsum, s), "residual sum");
        double rr = 0.0;
        HIP_TRY(hipMemcpyAsync(&rr, dsum, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
        HIP_TRY(hipStreamSynchronize(s), "sync");
        rel = nf > 0.0 ? std::sqrt(rr) / nf : std::sqrt(rr);
        if (rel <= rel_tol) {
            status = ST_OK;
            break;
        }
        if (cyc >= max_cycles) break;
        // V-cycle: down (pre-smooth, residual, restrict), coarsest, up
        // (prolongate, post-smooth)
        for (int l = 0; l + 1 < nlev; ++l) {
            HIP_TRY(zero(l), "memset");
            if ((rc = smooth(l, pre))) return rc;
            HIP_TRY(launch_mg_residual(f32, lv[l], e[l], R(l), RES(l), s), "mg residual");
            HIP_TRY(launch_mg_restrict(f32, lv[l], lv[l + 1], tabs[l], RES(l), R(l + 1),
                                       base + rtmp_off, s),
                    "mg restrict");
        }
        HIP_TRY(zero(nlev - 1), "memset");
        if ((rc = smooth(nlev - 1, coarse_sweeps))) return rc;
        for (int l = nlev - 2; l >= 0; --l) {
            HIP_TRY(launch_mg_prolong(f32, lv[l], lv[l + 1], tabs[l], e[l], e[l + 1], s),
                    "mg prolong");
            if ((rc = smooth(l, post))) return rc;
        }
        HIP_TRY(launch_correct(g, u, e[0], f32, s), "correct");
        ++cyc;
        if (smoother == 1) {
            rc = check_gs_status(s);
            if (rc) return rc;
        }
    }
    HIP_TRY(hipStreamSynchronize(s), "sync");
    if (cycles_done) *cycles_done = cyc;
    if (rel_res_out) *rel_res_out = rel;
    if (status == ST_ENOCONV) set_error("relative residual above rel_tol after max_cycles V-cycles");
    return status;
}

}  // extern "C"
