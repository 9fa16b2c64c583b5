// mg.hip -- geometric multigrid transfers and the level residual.
//
// Multigrid is the solver the smoothers of Sec. 3 exist for (Sec. 1); the
// V-cycle runs the fused Jacobi pass, the Gauss-Seidel wavefront or the
// red-black pass as its smoother on every level.  The kernels here are the
// glue between levels, all elementwise and HBM-bound:
//
//   * level residual   res = r - ((6*c) - s)         (precision of the level)
//   * restriction      r_c = scale * P^T res          (coarse right-hand side,
//                                                      one pass per axis)
//   * prolongation     e_f = e_f + P e_c              (trilinear interpolation)
//
// Levels: n interior points per axis at x_i = i/(n+1); the next level has
// nc = floor((n+1)/2) - 1.  Fine point i sits on the coarse grid at
// i (nc+1)/(n+1) = I0 + q/(n+1); its interpolation weights are
// wm = (n+1-q)/(n+1) on I0 and wq = q/(n+1) on I0+1 (one rounded division in
// the level's precision, coarse ghosts 0).  When n+1 is even this is the
// nested grid (weights 1, or 1/2 and 1/2; restriction = full weighting);
// otherwise (n = 512) the coarse spacing is slightly more than twice the fine
// one and the same formulas interpolate geometrically.  The per-axis tables
// (I0, wm, wq per fine point; the first and last fine point of every coarse
// point's support) are computed on the host in the level's precision and
// read by the kernels; no division happens on the device.
//
// Evaluation order (fixed; results are bit-identical from run to run):
// restriction sums x first (fine i increasing, acc = acc + w * r from 0),
// then y over those sums, then z, then multiplies by scale; prolongation
// interpolates along x, then y, then z, each (wm * lo) + (wq * hi).
#include <cmath>
#include <cstring>

#include "internal.h"

#pragma clang fp contract(off)

namespace stk {
namespace {

// Largest number of fine points with a non-zero weight towards one coarse
// point, per axis (nc + 1 = floor((n+1)/2) gives at most 4; the host checks).
constexpr int MG_MAXS = 5;

template <typename T>
struct MgAxisDev {
    const int *i0;   // [n + 1]: coarse index I0 of fine point i (entry 0 unused)
    const T *wm;     // [n + 1]: weight on I0
    const T *wq;     // [n + 1]: weight on I0 + 1
    const int *lo;   // [nc + 1]: first fine point with a non-zero weight on I
    const int *hi;   // [nc + 1]: last such point
};

template <typename T>
struct MgArgs {
    MgAxisDev<T> ax[3];
    int fnx, fny, fnz, fh;   // fine level interior extents and ghost width
    int64_t fpx, fplane;     // fine padded pitches
    int cnx, cny, cnz;       // coarse interior extents (ghost width 1)
    int64_t cpx, cplane;
    T scale;
};

// res = r - ((6*c) - s); e padded (ghost width h), r and res interior-only.
// One wave per row, four rows per block.
template <typename T>
__global__ void __launch_bounds__(256) mg_residual_kernel(const T *__restrict__ e,
                                                          const T *__restrict__ r,
                                                          T *__restrict__ res, int nx, int ny,
                                                          int h, int64_t px, int64_t plane) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rows_per_plane = (ny + 3) / 4;
    const int kz = blockIdx.x / rows_per_plane;
    const int jr = (blockIdx.x - kz * rows_per_plane) * 4 + w;
    if (jr >= ny) return;
    const T *c = e + (int64_t)(kz + h) * plane + (int64_t)(jr + h) * px + h;
    const int64_t fo = ((int64_t)kz * ny + jr) * nx;
    for (int i = lane; i < nx; i += 64) {
        T s = c[i - 1];
        s = s + c[i + 1];
        s = s + c[i - px];
        s = s + c[i + px];
        s = s + c[i - plane];
        s = s + c[i + plane];
        res[fo + i] = r[fo + i] - ((T(6) * c[i]) - s);
    }
}

// weight of fine point i towards coarse point I on one axis
template <typename T>
__device__ __forceinline__ T axis_w(const MgAxisDev<T> &a, int i, int I) {
    const int i0 = a.i0[i];
    return I == i0 ? a.wm[i] : (I == i0 + 1 ? a.wq[i] : T(0));
}

// r_c = scale * P^T res (both interior-only), as three one-axis passes that
// keep the evaluation order: the x sums of every fine row (X: fine z, fine
// y, coarse x), the y sums of those (Y: fine z, coarse y, coarse x), then the
// z sums times scale.  Each pass reads its input about once (a fine value
// lies in the support of at most two coarse points per axis), where one
// kernel gathering the whole 3-d support per coarse point read every fine
// residual about eight times through L2.
//
// x pass: one wave per run of MG_XR fine rows of one plane, lanes over coarse
// x; a lane reads its x weights once for the run.
constexpr int MG_XR = 8;
template <typename T>
__global__ void __launch_bounds__(256) mg_restrict_x_kernel(MgArgs<T> M,
                                                            const T *__restrict__ res,
                                                            T *__restrict__ X) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int runs = (M.fny + MG_XR - 1) / MG_XR;
    const int per_plane = (runs + 3) / 4;
    const int k = blockIdx.x / per_plane;  // fine plane, 0-based
    const int run = (blockIdx.x - k * per_plane) * 4 + w;
    if (run >= runs) return;
    const int j_lo = run * MG_XR, j_hi = min(j_lo + MG_XR, M.fny);  // fine rows, 0-based
    const MgAxisDev<T> &ax = M.ax[0];
    for (int I = lane + 1; I <= M.cnx; I += 64) {
        const int i0 = ax.lo[I], ni = ax.hi[I] - i0 + 1;
        T wx[MG_MAXS];
#pragma unroll
        for (int q = 0; q < MG_MAXS; ++q) wx[q] = q < ni ? axis_w(ax, i0 + q, I) : T(0);
        for (int j = j_lo; j < j_hi; ++j) {
            const T *row = res + ((int64_t)k * M.fny + j) * M.fnx + (i0 - 1);
            T xs = T(0);
#pragma unroll
            for (int a = 0; a < MG_MAXS; ++a) {
                if (a >= ni) break;
                xs = xs + (wx[a] * row[a]);
            }
            X[((int64_t)k * M.fny + j) * M.cnx + (I - 1)] = xs;
        }
    }
}

// y pass: one wave per (fine plane, coarse row), lanes over coarse x.
template <typename T>
__global__ void __launch_bounds__(256) mg_restrict_y_kernel(MgArgs<T> M,
                                                            const T *__restrict__ X,
                                                            T *__restrict__ Y) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rows_per_plane = (M.cny + 3) / 4;
    const int k = blockIdx.x / rows_per_plane;  // fine plane, 0-based
    const int J = (blockIdx.x - k * rows_per_plane) * 4 + w + 1;
    if (J > M.cny) return;
    const MgAxisDev<T> &ay = M.ax[1];
    const int j0 = ay.lo[J], nj = ay.hi[J] - j0 + 1;
    T wy[MG_MAXS];
#pragma unroll
    for (int q = 0; q < MG_MAXS; ++q) wy[q] = q < nj ? axis_w(ay, j0 + q, J) : T(0);
    const T *xin = X + ((int64_t)k * M.fny + (j0 - 1)) * M.cnx;
    T *out = Y + ((int64_t)k * M.cny + (J - 1)) * M.cnx;
    for (int I = lane; I < M.cnx; I += 64) {
        T ys = T(0);
#pragma unroll
        for (int b = 0; b < MG_MAXS; ++b) {
            if (b >= nj) break;
            ys = ys + (wy[b] * xin[(int64_t)b * M.cnx + I]);
        }
        out[I] = ys;
    }
}

// z pass: one wave per coarse row (K, J), lanes over coarse x.
template <typename T>
__global__ void __launch_bounds__(256) mg_restrict_z_kernel(MgArgs<T> M,
                                                            const T *__restrict__ Y,
                                                            T *__restrict__ rc) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rows_per_plane = (M.cny + 3) / 4;
    const int K = blockIdx.x / rows_per_plane + 1;
    const int J = (blockIdx.x - (K - 1) * rows_per_plane) * 4 + w + 1;
    if (J > M.cny) return;
    const MgAxisDev<T> &az = M.ax[2];
    const int k0 = az.lo[K], nk = az.hi[K] - k0 + 1;
    T wz[MG_MAXS];
#pragma unroll
    for (int q = 0; q < MG_MAXS; ++q) wz[q] = q < nk ? axis_w(az, k0 + q, K) : T(0);
    const int64_t zstride = (int64_t)M.cny * M.cnx;
    const T *yin = Y + ((int64_t)(k0 - 1) * M.cny + (J - 1)) * M.cnx;
    T *out = rc + ((int64_t)(K - 1) * M.cny + (J - 1)) * M.cnx;
    for (int I = lane; I < M.cnx; I += 64) {
        T zs = T(0);
#pragma unroll
        for (int c = 0; c < MG_MAXS; ++c) {
            if (c >= nk) break;
            zs = zs + (wz[c] * yin[c * zstride + I]);
        }
        out[I] = zs * M.scale;
    }
}

// e_f += P e_c; e_f padded (ghost width fh), e_c padded (ghost width 1, ghosts
// 0).  One wave per fine row.
template <typename T>
__global__ void __launch_bounds__(256) mg_prolong_kernel(MgArgs<T> M, T *__restrict__ ef,
                                                         const T *__restrict__ ec) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int rows_per_plane = (M.fny + 3) / 4;
    const int k = blockIdx.x / rows_per_plane + 1;
    const int j = (blockIdx.x - (k - 1) * rows_per_plane) * 4 + w + 1;
    if (j > M.fny) return;
    const MgAxisDev<T> &ax = M.ax[0], &ay = M.ax[1], &az = M.ax[2];
    const int J0 = ay.i0[j], K0 = az.i0[k];
    const T wmy = ay.wm[j], wqy = ay.wq[j], wmz = az.wm[k], wqz = az.wq[k];
    T *out = ef + (int64_t)(k - 1 + M.fh) * M.fplane + (int64_t)(j - 1 + M.fh) * M.fpx +
             (M.fh - 1);
    // unrolled so that several points' table and coarse loads are in flight
#pragma unroll 4
    for (int i = lane + 1; i <= M.fnx; i += 64) {
        const int I0 = ax.i0[i];
        const T wmx = ax.wm[i], wqx = ax.wq[i];
        T vy[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            T vx[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const T *row = ec + (int64_t)(K0 + c) * M.cplane + (int64_t)(J0 + b) * M.cpx;
                vx[b] = (wmx * row[I0]) + (wqx * row[I0 + 1]);
            }
            vy[c] = (wmy * vx[0]) + (wqy * vx[1]);
        }
        const T v = (wmz * vy[0]) + (wqz * vy[1]);
        out[i] = out[i] + v;
    }
}

template <typename T>
MgArgs<T> make_mg_args(const Geom &fine, const Geom &coarse, const MgTables &tab, double scale) {
    MgArgs<T> M;
    for (int d = 0; d < 3; ++d) {
        const unsigned char *b = static_cast<const unsigned char *>(tab.dev);
        M.ax[d].i0 = reinterpret_cast<const int *>(b + tab.off_i0[d]);
        M.ax[d].wm = reinterpret_cast<const T *>(b + tab.off_wm[d]);
        M.ax[d].wq = reinterpret_cast<const T *>(b + tab.off_wq[d]);
        M.ax[d].lo = reinterpret_cast<const int *>(b + tab.off_lo[d]);
        M.ax[d].hi = reinterpret_cast<const int *>(b + tab.off_hi[d]);
    }
    M.fnx = fine.nx; M.fny = fine.ny; M.fnz = fine.nz; M.fh = fine.h;
    M.fpx = fine.px; M.fplane = fine.plane();
    M.cnx = coarse.nx; M.cny = coarse.ny; M.cnz = coarse.nz;
    M.cpx = coarse.px; M.cplane = coarse.plane();
    M.scale = (T)scale;
    return M;
}

// Host tables of one axis in precision T, appended to `bytes`.  False if a
// coarse point's support exceeds MG_MAXS fine points (never for
// nc + 1 = floor((n+1)/2), where it is at most 4).
template <typename T>
bool axis_tables(int n, int nc, std::vector<unsigned char> &bytes, size_t off[5]) {
    auto put = [&](const void *p, size_t nbytes) {
        const size_t o = (bytes.size() + 255) / 256 * 256;
        bytes.resize(o + nbytes);
        std::memcpy(bytes.data() + o, p, nbytes);
        return o;
    };
    std::vector<int> i0(n + 1, 0), lo(nc + 1, 0), hi(nc + 1, 0);
    std::vector<T> wm(n + 1, T(0)), wq(n + 1, T(0));
    for (int i = 1; i <= n; ++i) {
        const int64_t p = (int64_t)i * (nc + 1);
        const int64_t a = p / (n + 1), q = p % (n + 1);
        i0[i] = (int)a;
        wm[i] = (T)(n + 1 - q) / (T)(n + 1);
        wq[i] = (T)q / (T)(n + 1);
    }
    for (int I = 1; I <= nc; ++I) {
        int64_t l = ((int64_t)(I - 1) * (n + 1)) / (nc + 1) + 1;
        int64_t h = ((int64_t)(I + 1) * (n + 1) - 1) / (nc + 1);
        lo[I] = (int)(l < 1 ? 1 : l);
        hi[I] = (int)(h > n ? n : h);
        if (hi[I] - lo[I] + 1 > MG_MAXS) return false;
    }
    off[0] = put(i0.data(), i0.size() * sizeof(int));
    off[1] = put(wm.data(), wm.size() * sizeof(T));
    off[2] = put(wq.data(), wq.size() * sizeof(T));
    off[3] = put(lo.data(), lo.size() * sizeof(int));
    off[4] = put(hi.data(), hi.size() * sizeof(int));
    return true;
}

}  // namespace

int mg_coarse_n(int n) { return (n + 1) / 2 - 1; }

double mg_scale(const Geom &g) {
    const double rx = (double)(mg_coarse_n(g.nx) + 1) / (double)(g.nx + 1);
    const double ry = (double)(mg_coarse_n(g.ny) + 1) / (double)(g.ny + 1);
    const double rz = (double)(mg_coarse_n(g.nz) + 1) / (double)(g.nz + 1);
    if (rx == ry && ry == rz) return rx;
    return std::cbrt(rx * ry * rz);
}

bool mg_build_tables(bool fp32, const Geom &fine, std::vector<unsigned char> &bytes,
                     MgTables &tab) {
    const int n[3] = {fine.nx, fine.ny, fine.nz};
    for (int d = 0; d < 3; ++d) {
        size_t off[5];
        const bool ok = fp32 ? axis_tables<float>(n[d], mg_coarse_n(n[d]), bytes, off)
                             : axis_tables<double>(n[d], mg_coarse_n(n[d]), bytes, off);
        if (!ok) return false;
        tab.off_i0[d] = off[0];
        tab.off_wm[d] = off[1];
        tab.off_wq[d] = off[2];
        tab.off_lo[d] = off[3];
        tab.off_hi[d] = off[4];
    }
    return true;
}

static unsigned rows_grid(int ny, int nz) { return (unsigned)((int64_t)nz * ((ny + 3) / 4)); }

hipError_t launch_mg_residual(bool fp32, const Geom &g, const void *e, const void *r, void *res,
                              hipStream_t s) {
    if (fp32)
        hipLaunchKernelGGL(mg_residual_kernel<float>, dim3(rows_grid(g.ny, g.nz)), dim3(256), 0, s,
                           (const float *)e, (const float *)r, (float *)res, g.nx, g.ny, g.h, g.px,
                           g.plane());
    else
        hipLaunchKernelGGL(mg_residual_kernel<double>, dim3(rows_grid(g.ny, g.nz)), dim3(256), 0,
                           s, (const double *)e, (const double *)r, (double *)res, g.nx, g.ny, g.h,
                           g.px, g.plane());
    return hipGetLastError();
}

size_t mg_restrict_tmp_bytes(bool fp32, const Geom &fine, const Geom &coarse) {
    const size_t x = (size_t)fine.nz * fine.ny * coarse.nx, y = (size_t)fine.nz * coarse.ny * coarse.nx;
    return (x + y) * (fp32 ? sizeof(float) : sizeof(double));
}

template <typename T>
hipError_t restrict_t(const Geom &fine, const Geom &coarse, const MgTables &tab, const T *res,
                      T *rc, T *tmp, hipStream_t s) {
    const MgArgs<T> M = make_mg_args<T>(fine, coarse, tab, mg_scale(fine));
    T *X = tmp;
    T *Y = tmp + (size_t)fine.nz * fine.ny * coarse.nx;
    const int runs = (fine.ny + MG_XR - 1) / MG_XR;
    hipLaunchKernelGGL(mg_restrict_x_kernel<T>, dim3((unsigned)fine.nz * ((runs + 3) / 4)),
                       dim3(256), 0, s, M, res, X);
    hipLaunchKernelGGL(mg_restrict_y_kernel<T>, dim3(rows_grid(coarse.ny, fine.nz)), dim3(256), 0,
                       s, M, (const T *)X, Y);
    hipLaunchKernelGGL(mg_restrict_z_kernel<T>, dim3(rows_grid(coarse.ny, coarse.nz)), dim3(256),
                       0, s, M, (const T *)Y, rc);
    return hipGetLastError();
}

hipError_t launch_mg_restrict(bool fp32, const Geom &fine, const Geom &coarse,
                              const MgTables &tab, const void *res, void *rc, void *tmp,
                              hipStream_t s) {
    if (fp32)
        return restrict_t<float>(fine, coarse, tab, (const float *)res, (float *)rc, (float *)tmp,
                                 s);
    return restrict_t<double>(fine, coarse, tab, (const double *)res, (double *)rc,
                              (double *)tmp, s);
}

hipError_t launch_mg_prolong(bool fp32, const Geom &fine, const Geom &coarse, const MgTables &tab,
                             void *ef, const void *ec, hipStream_t s) {
    const dim3 grid(rows_grid(fine.ny, fine.nz));
    if (fp32)
        hipLaunchKernelGGL(mg_prolong_kernel<float>, grid, dim3(256), 0, s,
                           make_mg_args<float>(fine, coarse, tab, 1.0), (float *)ef,
                           (const float *)ec);
    else
        hipLaunchKernelGGL(mg_prolong_kernel<double>, grid, dim3(256), 0, s,
                           make_mg_args<double>(fine, coarse, tab, 1.0), (double *)ef,
                           (const double *)ec);
    return hipGetLastError();
}

}  // namespace stk
