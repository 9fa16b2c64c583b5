// internal.h -- declarations shared by the HIP kernels and the host runtime of
// libstencil.  Not part of the public ABI (include/stencil.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace stk {

// Grid geometry in elements (padded layout, x contiguous).
struct Geom {
    int nx, ny, nz, h;
    int64_t px, py, pz;  // padded extents
    int64_t plane() const { return px * py; }
    int64_t count() const { return px * py * pz; }
    int64_t interior() const { return (int64_t)nx * ny * nz; }
};

// Per-(dtype, TB) tile configuration of the fused Jacobi pass.
struct JacTileCfg {
    int tb;     // time levels kept on chip (sweeps per pass)
    int vx;     // x points per lane (16-byte vectors when vx * sizeof(T) == 16)
    int ry;     // rows per wave
    int nw;     // waves per workgroup
    int tx() const { return 64 * vx; }
    int ty() const { return nw * ry; }
    int ow() const { return tx() - 2 * tb - (vx - 1); }  // output tile width
    int oh() const { return ty() - 2 * tb; }             // output tile height
};

JacTileCfg jacobi_tile_cfg(bool fp32, int tb, bool has_f);
// x-y tiles of one fused pass over g, and how many take the unmasked path.
void jacobi_tile_count(bool fp32, int tb, bool has_f, const Geom &g, int *tiles, int *interior);

// One fused Jacobi pass: dst <- TB sweeps of src (interior only).
// zc = output planes per z-chunk (0 = planner choice).
hipError_t launch_jacobi_pass(bool fp32, int tb, const Geom &g, const void *src, void *dst,
                              const void *f, double a, double b, double gw, int zc,
                              hipStream_t s);

// One grid of a batched pass (job service).
struct JacBatchItem {
    Geom g;
    const void *src;
    void *dst;
    const void *f;
    double a, b, gw;
};
size_t jacobi_batch_table_bytes(int njobs);
// All items share dtype, tb and the presence of the centre / RHS terms.
// table_dev: device buffer of jacobi_batch_table_bytes(items.size()) bytes;
// host_buf: staging memory that must stay untouched until the copy is done
// (the copy is from pageable memory, so it is complete when the call returns).
hipError_t launch_jacobi_batch(bool fp32, int tb, bool has_a, bool has_f,
                               const std::vector<JacBatchItem> &items, void *table_dev,
                               std::vector<unsigned char> &host_buf, hipStream_t s);

// One fused red-black Gauss-Seidel pass: dst <- sweeps (1..4) red-black
// sweeps of src, as 2*sweeps levels of the fused pass.
hipError_t launch_rbgs_pass(bool fp32, int sweeps, const Geom &g, const void *src, void *dst,
                            const void *f, double a, double b, double gw, hipStream_t s);

// The fused pass for one level count TB (1..8); each TB is compiled in its
// own translation unit, the functions above dispatch on tb.
template <int TB>
struct JacobiLevels {
    static JacTileCfg cfg(bool fp32, bool has_f);
    static void tiles(bool fp32, bool has_f, const Geom &g, int *tiles, int *interior);
    static hipError_t pass(bool fp32, const Geom &g, const void *src, void *dst, const void *f,
                           double a, double b, double gw, int zc, hipStream_t s);
    // red-black Gauss-Seidel: TB/2 sweeps in one pass (TB even)
    static hipError_t rb_pass(bool fp32, const Geom &g, const void *src, void *dst,
                              const void *f, double a, double b, double gw, hipStream_t s);
    static hipError_t batch(bool fp32, bool has_a, bool has_f,
                            const std::vector<JacBatchItem> &items, void *table_dev,
                            std::vector<unsigned char> &host_buf, hipStream_t s);
    static size_t table_bytes(int njobs);
};

// Ghost-layer helpers (all ghost cells of a padded grid).
hipError_t launch_fill_ghosts(bool fp32, const Geom &g, void *u, double value, hipStream_t s);
hipError_t launch_copy_ghosts(bool fp32, const Geom &g, const void *src, void *dst,
                              hipStream_t s);
hipError_t launch_copy_interior(bool fp32, const Geom &g, const void *src, void *dst,
                                hipStream_t s);
hipError_t launch_zero(void *p, int64_t bytes, hipStream_t s);

// FP64 residual r = f' - ((6c) - s) as double and/or float, with per-block
// partial sums of r^2 written to partials[nblocks]; returns nblocks.
hipError_t launch_residual_poisson(const Geom &g, const double *u, const double *fp, double *r64,
                                   float *r32, double *partials, int *nblocks, hipStream_t s);
// Generic defect r = (one update of u) - c (FP64), written as float and/or double.
hipError_t launch_defect(const Geom &g, const double *u, const double *f, double a, double b,
                         double gw, double *r64, float *r32, hipStream_t s);
// Deterministic fixed-tree sum of partials[n] into out[0].
hipError_t launch_sum_partials(const double *partials, int n, double *out, hipStream_t s);
int residual_partial_count(const Geom &g);
// u(interior) += (double)e(interior); e padded float or double grid of same geometry.
hipError_t launch_correct(const Geom &g, double *u, const void *e, bool e_fp32, hipStream_t s);

// Gauss-Seidel wavefront: one launch with all `sweeps` (1..4095) in flight.
// Its workspace (progress counters, ticket, item table) is taken with
// hipMallocAsync on s and released with hipFreeAsync after the launch.
hipError_t launch_gs(bool fp32, const Geom &g, void *u, const void *f, double a, double b,
                     double gw, int sweeps, hipStream_t s);
// Allocation-free variant: the workspace lives in a static device array of
// GS_NOALLOC_BYTES per device instead of the stream-ordered allocator.
// hipErrorInvalidValue when the workspace of `sweeps` does not fit it.
constexpr size_t GS_NOALLOC_BYTES = (size_t)4 << 20;
size_t gs_workspace_bytes(int sweeps, int ny, int nz);
hipError_t launch_gs_noalloc(bool fp32, const Geom &g, void *u, const void *f, double a,
                             double b, double gw, int sweeps, hipStream_t s);
// Synchronizes s, then reads (and optionally clears, with the abort word)
// the device's wavefront status: bit 0 = a launch gave up waiting.
hipError_t gs_status(int dev, hipStream_t s, bool clear, uint32_t *status);
// Raises the device's abort word (running and later wavefront launches give
// up at their next wait) until gs_status clears it.
hipError_t gs_abort(int dev);
// Polls of one wavefront wait before it gives up (0 = the default, 2^24).
void gs_set_spin_limit(uint32_t polls);

// Batched wavefront (job service): `sweeps` sweeps of every item's grid in
// one launch; items of all grids share one ticket counter in key order.
struct GsBatchItem {
    Geom g;
    void *u;
    const void *f;
    double a, b, gw;
    int sweeps;
};
// Device workspace (job table, item list, counters) owned by the caller;
// must not be reused before the launch that used it has completed.
struct GsBatchWork {
    void *dev = nullptr;
    size_t dev_bytes = 0;
    std::vector<uint64_t> items;
    std::vector<unsigned char> jobs_host;
    ~GsBatchWork();
};
hipError_t launch_gs_batch(bool fp32, bool has_a, bool has_f,
                           const std::vector<GsBatchItem> &items, GsBatchWork &w, hipStream_t s);

// ---- geometric multigrid (mg.hip) ----
// Next coarser level: floor((n+1)/2) - 1 interior points per axis.
int mg_coarse_n(int n);
// h/H factor of the restriction from level g to the next (FP64, host).
double mg_scale(const Geom &g);
// Per-axis transfer tables between level `fine` and the next one, in the
// level's precision: appended to `bytes` (host), offsets in `tab`; the caller
// copies `bytes` to the device and sets tab.dev.
struct MgTables {
    void *dev = nullptr;
    size_t off_i0[3], off_wm[3], off_wq[3], off_lo[3], off_hi[3];
};
bool mg_build_tables(bool fp32, const Geom &fine, std::vector<unsigned char> &bytes,
                     MgTables &tab);
// res = r - ((6*c) - s) (e padded; r, res interior-only).
hipError_t launch_mg_residual(bool fp32, const Geom &g, const void *e, const void *r, void *res,
                              hipStream_t s);
// rc = scale * P^T res (interior-only; coarse has ghost width 1).  tmp:
// device workspace of mg_restrict_tmp_bytes(fp32, fine, coarse) bytes for
// the per-axis partial sums.
size_t mg_restrict_tmp_bytes(bool fp32, const Geom &fine, const Geom &coarse);
hipError_t launch_mg_restrict(bool fp32, const Geom &fine, const Geom &coarse,
                              const MgTables &tab, const void *res, void *rc, void *tmp,
                              hipStream_t s);
// ef += P ec (both padded).
hipError_t launch_mg_prolong(bool fp32, const Geom &fine, const Geom &coarse, const MgTables &tab,
                             void *ef, const void *ec, hipStream_t s);

// Thread-local error message used by the C ABI.
void set_error(const std::string &msg);

}  // namespace stk
