// aux.hip -- ghost-layer maintenance, FP64 residual / defect with a
// deterministic reduction, and the FP64 correction of the refinement loop.
#include "internal.h"

#pragma clang fp contract(off)

namespace stk {
namespace {

// Ghost layer of a padded grid in two parts.  Blocks [0, nfull) take the
// rows that lie entirely in the ghost layer (z ghost planes, then the y ghost
// rows of interior planes), one 64-lane wave per row.  The remaining blocks
// take the 2h x ghosts of every interior row, one element per thread, so the
// interior rows cost no idle waves.
template <typename T, bool COPY>
__global__ void __launch_bounds__(256) ghost_kernel(T *__restrict__ dst, const T *__restrict__ src,
                                                    T value, int64_t px, int64_t py, int64_t pz,
                                                    int h, int64_t nfull) {
    const int64_t zrows = 2 * h * py;          // rows of the 2h ghost planes
    const int64_t nyi = py - 2 * h, nzi = pz - 2 * h;
    if ((int64_t)blockIdx.x < nfull) {
        const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
        int64_t k, j;
        if (r < zrows) {
            const int64_t pl = r / py;                   // 0 .. 2h-1
            k = pl < h ? pl : pz - 2 * h + pl;
            j = r - pl * py;
        } else {
            const int64_t q = r - zrows;                 // y ghost rows of interior planes
            if (q >= 2 * h * nzi) return;
            const int64_t kk = q / (2 * h), jj = q - kk * (2 * h);
            k = h + kk;
            j = jj < h ? jj : py - 2 * h + jj;
        }
        const int64_t base = (k * py + j) * px;
        for (int64_t i = threadIdx.x & 63; i < px; i += 64)
            dst[base + i] = COPY ? src[base + i] : value;
    } else {
        const int64_t e = ((int64_t)blockIdx.x - nfull) * 256 + threadIdx.x;
        if (e >= nzi * nyi * 2 * h) return;
        const int64_t row = e / (2 * h);
        const int i = (int)(e - row * (2 * h));
        const int64_t k = h + row / nyi, j = h + row % nyi;
        const int64_t x = i < h ? i : px - 2 * h + i;
        const int64_t o = (k * py + j) * px + x;
        dst[o] = COPY ? src[o] : value;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    // fixed butterfly order: the result is identical on every run
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}

// r = f' - ((6*c) - s) on interior rows; 4 rows (one per wave) per block.
// Each block writes the sum of its r^2 to partials[blockIdx.x].  u == nullptr
// stands for the zero grid (r = f' exactly), which gives ||f'|| with the same
// reduction order without a zero grid in memory.
__global__ void __launch_bounds__(256) residual_kernel(const double *__restrict__ u,
                                                       const double *__restrict__ fp,
                                                       double *__restrict__ r64,
                                                       float *__restrict__ r32,
                                                       double *__restrict__ partials, int nx,
                                                       int ny, int nz, int h, int64_t px,
                                                       int64_t plane) {
    __shared__ double red[4];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rows_per_plane = (ny + 3) / 4;
    const int kz = blockIdx.x / rows_per_plane;
    const int jr = (blockIdx.x - kz * rows_per_plane) * 4 + w;
    double acc = 0.0;
    if (jr < ny) {
        const int k = kz + h, j = jr + h;
        const int64_t fo = ((int64_t)kz * ny + jr) * nx;
        if (!u) {
            for (int i = lane; i < nx; i += 64) {
                const double rv = fp ? fp[fo + i] : 0.0;
                if (r64) r64[fo + i] = rv;
                if (r32) r32[fo + i] = (float)rv;
                acc = acc + rv * rv;
            }
        }
        const double *c = u ? u + (int64_t)k * plane + (int64_t)j * px + h : nullptr;
        for (int i = lane; c && i < nx; i += 64) {
            double s = c[i - 1];
            s = s + c[i + 1];
            s = s + c[i - px];
            s = s + c[i + px];
            s = s + c[i - plane];
            s = s + c[i + plane];
            const double fv = fp ? fp[fo + i] : 0.0;
            const double rv = fv - ((6.0 * c[i]) - s);
            if (r64) r64[fo + i] = rv;
            if (r32) r32[fo + i] = (float)rv;
            acc = acc + rv * rv;
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) red[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// r = (one update of u) - c, FP64.
__global__ void __launch_bounds__(256) defect_kernel(const double *__restrict__ u,
                                                     const double *__restrict__ f, double a,
                                                     double b, double g, double *__restrict__ r64,
                                                     float *__restrict__ r32, int nx, int ny,
                                                     int nz, int h, int64_t px, int64_t plane) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rows_per_plane = (ny + 3) / 4;
    const int kz = blockIdx.x / rows_per_plane;
    const int jr = (blockIdx.x - kz * rows_per_plane) * 4 + w;
    if (jr >= ny) return;
    const int k = kz + h, j = jr + h;
    const double *c = u + (int64_t)k * plane + (int64_t)j * px + h;
    const int64_t fo = ((int64_t)kz * ny + jr) * nx;
    for (int i = lane; i < nx; i += 64) {
        double s = c[i - 1];
        s = s + c[i + 1];
        s = s + c[i - px];
        s = s + c[i + px];
        s = s + c[i - plane];
        s = s + c[i + plane];
        double v = (a != 0.0) ? (a * c[i]) + (b * s) : b * s;
        if (f) v = v + (g * f[fo + i]);
        const double rv = v - c[i];
        if (r64) r64[fo + i] = rv;
        if (r32) r32[fo + i] = (float)rv;
    }
}

// Fixed-order sum of n partials: thread t sums t, t+1024, ... sequentially,
// then a fixed tree over the 1024 thread sums.
__global__ void __launch_bounds__(1024) sum_kernel(const double *__restrict__ p, int n,
                                                   double *__restrict__ out) {
    __shared__ double red[16];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) acc = acc + p[i];
    acc = wave_sum(acc);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 16; ++i) t = t + red[i];
        out[0] = t;
    }
}

template <typename E>
__global__ void __launch_bounds__(256) correct_kernel(double *__restrict__ u,
                                                      const E *__restrict__ e, int nx, int ny,
                                                      int nz, int h, int64_t px, int64_t plane) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rows_per_plane = (ny + 3) / 4;
    const int kz = blockIdx.x / rows_per_plane;
    const int jr = (blockIdx.x - kz * rows_per_plane) * 4 + w;
    if (jr >= ny) return;
    const int64_t o = (int64_t)(kz + h) * plane + (int64_t)(jr + h) * px + h;
    for (int i = lane; i < nx; i += 64) u[o + i] = u[o + i] + (double)e[o + i];
}

int row_blocks(const Geom &g) { return g.nz * ((g.ny + 3) / 4); }

}  // namespace

namespace {
struct GhostGrid {
    dim3 grid;
    int64_t nfull;
};
GhostGrid ghost_grid(const Geom &g) {
    const int64_t full_rows = 2 * g.h * g.py + 2 * g.h * (g.pz - 2 * g.h);
    const int64_t xg = (g.pz - 2 * g.h) * (g.py - 2 * g.h) * 2 * g.h;
    const int64_t nfull = (full_rows + 3) / 4;
    return GhostGrid{dim3((unsigned)(nfull + (xg + 255) / 256)), nfull};
}
}  // namespace

hipError_t launch_fill_ghosts(bool fp32, const Geom &g, void *u, double value, hipStream_t s) {
    const GhostGrid q = ghost_grid(g);
    if (fp32)
        hipLaunchKernelGGL((ghost_kernel<float, false>), q.grid, dim3(256), 0, s, (float *)u,
                           (const float *)nullptr, (float)value, g.px, g.py, g.pz, g.h, q.nfull);
    else
        hipLaunchKernelGGL((ghost_kernel<double, false>), q.grid, dim3(256), 0, s, (double *)u,
                           (const double *)nullptr, value, g.px, g.py, g.pz, g.h, q.nfull);
    return hipGetLastError();
}

hipError_t launch_copy_ghosts(bool fp32, const Geom &g, const void *src, void *dst,
                              hipStream_t s) {
    const GhostGrid q = ghost_grid(g);
    if (fp32)
        hipLaunchKernelGGL((ghost_kernel<float, true>), q.grid, dim3(256), 0, s, (float *)dst,
                           (const float *)src, 0.0f, g.px, g.py, g.pz, g.h, q.nfull);
    else
        hipLaunchKernelGGL((ghost_kernel<double, true>), q.grid, dim3(256), 0, s, (double *)dst,
                           (const double *)src, 0.0, g.px, g.py, g.pz, g.h, q.nfull);
    return hipGetLastError();
}

hipError_t launch_copy_interior(bool fp32, const Geom &g, const void *src, void *dst,
                                hipStream_t s) {
    // ghosts of src and dst are identical here, so a whole-array copy is exact
    return hipMemcpyAsync(dst, src, (size_t)g.count() * (fp32 ? 4 : 8), hipMemcpyDeviceToDevice,
                          s);
}

hipError_t launch_zero(void *p, int64_t bytes, hipStream_t s) {
    return hipMemsetAsync(p, 0, (size_t)bytes, s);
}

int residual_partial_count(const Geom &g) { return row_blocks(g); }

hipError_t launch_residual_poisson(const Geom &g, const double *u, const double *fp, double *r64,
                                   float *r32, double *partials, int *nblocks, hipStream_t s) {
    const int nb = row_blocks(g);
    hipLaunchKernelGGL(residual_kernel, dim3(nb), dim3(256), 0, s, u, fp, r64, r32, partials,
                       g.nx, g.ny, g.nz, g.h, g.px, g.plane());
    if (nblocks) *nblocks = nb;
    return hipGetLastError();
}

hipError_t launch_defect(const Geom &g, const double *u, const double *f, double a, double b,
                         double gw, double *r64, float *r32, hipStream_t s) {
    hipLaunchKernelGGL(defect_kernel, dim3(row_blocks(g)), dim3(256), 0, s, u, f, a, b, gw, r64,
                       r32, g.nx, g.ny, g.nz, g.h, g.px, g.plane());
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *partials, int n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1024), 0, s, partials, n, out);
    return hipGetLastError();
}

hipError_t launch_correct(const Geom &g, double *u, const void *e, bool e_fp32, hipStream_t s) {
    if (e_fp32)
        hipLaunchKernelGGL((correct_kernel<float>), dim3(row_blocks(g)), dim3(256), 0, s, u,
                           (const float *)e, g.nx, g.ny, g.nz, g.h, g.px, g.plane());
    else
        hipLaunchKernelGGL((correct_kernel<double>), dim3(row_blocks(g)), dim3(256), 0, s, u,
                           (const double *)e, g.nx, g.ny, g.nz, g.h, g.px, g.plane());
    return hipGetLastError();
}

}  // namespace stk
