// jacobi_impl.h -- fused multi-sweep Jacobi pass (gfx950): kernels and
// launchers.  Each level count TB is instantiated in its own translation
// unit (jacobi_t<TB>.hip) so that the builds run in parallel.
//
// Method (Sec. 3 Jacobi loop nest; Sec. 4 temporal wavefront blocking):
// TB consecutive Jacobi sweeps are applied in ONE pass over HBM.  The paper
// gives each of t threads sharing a cache one sweep, shifted in z, with a
// barrier after every plane.  Here one workgroup owns an x-y tile of the grid
// and marches it through z; the TB time levels of the tile live on chip:
//
//   * a wave covers 64*VX consecutive x sites (one 16-byte load per row when
//     VX*sizeof(T) == 16) and RY rows; NW waves stack in y, so a tile is
//     (64*VX) x (NW*RY) sites;
//   * level tau of plane p needs level tau-1 at planes p-1, p, p+1.  With a
//     skew of one plane per level, step s loads plane s of level 0 and
//     produces plane s-tau of level tau.  Each level keeps its two newest
//     planes in registers (centre plane and z-1 neighbour); the plane the
//     level below produces in the same step supplies z+;
//   * x neighbours come from adjacent lanes through DPP wave shifts, y
//     neighbours from the thread's own rows or, at wave edges, through a
//     small double-buffered LDS exchange (one barrier per step for all
//     levels);
//   * tiles overlap by TB sites on each side (the dependency cone), so only
//     the centre (64*VX - 2*TB - VX + 1) x (NW*RY - 2*TB) sites are stored;
//     ghost cells inside a tile keep their Dirichlet value at every level;
//   * z is split into chunks; a chunk starts TB planes early to fill the
//     pipeline (or at the ghost plane, where all levels are known).
//
// The same pass runs red-black Gauss-Seidel (RB = true): see jacobi_tile.
//
// HBM sees one load of level 0 and one store of level TB per site per pass:
// 2*sizeof(T) bytes per site per TB sweeps (Eq. (1) with the traffic divided
// by the number of fused sweeps).  All arithmetic keeps the canonical order
//   s = ((((x- + x+) + y-) + y+) + z-) + z+,  v = (a*c) + (b*s) [+ g*f]
// without FMA contraction, so every TB gives results bit-identical to TB
// sequential sweeps.
#pragma once
#include <atomic>
#include <type_traits>

#include "internal.h"

#pragma clang fp contract(off)

namespace stk {
namespace {

template <typename T, int VX>
struct VecT;
template <>
struct VecT<double, 2> {
    typedef double type __attribute__((ext_vector_type(2), aligned(8)));
};
template <>
struct VecT<float, 4> {
    typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct VecT<float, 2> {
    typedef float type __attribute__((ext_vector_type(2), aligned(4)));
};

__device__ __forceinline__ float from_lower_lane(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_upper_lane(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double from_lower_lane(double v) {
    int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_upper_lane(double v) {
    int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

template <typename T>
struct JacArgs {
    const T *src;
    T *dst;
    const T *f;      // interior-only right-hand side or nullptr
    int64_t px;      // row pitch (elements)
    int64_t plane;   // plane pitch (elements)
    int nx, ny, nz, h;
    T a, b, g;
    int tiles_x, tiles_y, nchunks, zc, ow, oh, ntiles;
};

typedef unsigned U32x2 __attribute__((ext_vector_type(2)));

template <typename T, int VX, bool EDGE>
__device__ __forceinline__ void load_row(const T *__restrict__ p, unsigned okmask, T (&out)[VX]) {
    if constexpr (!EDGE && (VX * sizeof(T) == 16 || (VX == 2 && sizeof(T) == 4))) {
        typedef typename VecT<T, VX>::type V;
        V v = *reinterpret_cast<const V *>(p);
#pragma unroll
        for (int i = 0; i < VX; ++i) out[i] = v[i];
    } else if constexpr (!EDGE) {
#pragma unroll
        for (int i = 0; i < VX; ++i) out[i] = p[i];
    } else {
#pragma unroll
        for (int i = 0; i < VX; ++i) out[i] = (okmask >> i & 1u) ? p[i] : T(0);
    }
}

template <typename T, int VX>
__device__ __forceinline__ void store_row(T *__restrict__ p, unsigned mask, const T (&v)[VX]) {
    constexpr unsigned full = (1u << VX) - 1u;
    if constexpr (VX * sizeof(T) == 16 || (VX == 2 && sizeof(T) == 4)) {
        if (mask == full) {
            typedef typename VecT<T, VX>::type V;
            V w;
#pragma unroll
            for (int i = 0; i < VX; ++i) w[i] = v[i];
            *reinterpret_cast<V *>(p) = w;
            return;
        }
    }
#pragma unroll
    for (int i = 0; i < VX; ++i)
        if (mask >> i & 1u) p[i] = v[i];
}

// Right-hand side ring: each thread keeps the f values of its own sites for
// planes s-2 .. s-TB (needed by levels 2..TB at step s) in LDS, so f is read
// from memory once per pass instead of once per level.  Used where it fits
// next to the exchange buffer in the 160 KB of LDS.
template <typename T, int TB, int VX, int RY, int NW, bool HAS_F>
struct FRing {
    static constexpr size_t xch_bytes = (size_t)2 * TB * NW * 2 * 64 * VX * sizeof(T);
    static constexpr size_t ring_elems = (size_t)(TB > 1 ? TB - 1 : 0) * RY * VX * NW * 64;
    static constexpr bool on =
        HAS_F && TB >= 2 && xch_bytes + ring_elems * sizeof(T) <= 160 * 1024;
    static constexpr size_t alloc = on ? ring_elems : 1;
};

// Ghost reset of one row: on the lanes of `mask` (all lanes for a ghost row,
// the ghost-column lanes otherwise, none for most rows) level k's new plane
// takes the value of level k-1, for k = 1..TB-1.  The exec mask and the skip
// branch live inside one asm statement, so the compiler sees in-place updates
// only: with the branch at the source level the register allocator changed
// the steady loop's register assignment and copied the prefetched plane at
// the loop's back edge, waiting there for loads issued one step earlier.
template <typename T, int TB, int RY, int VX>
__device__ __forceinline__ void ghost_reset_row(T (&Bb)[TB][RY][VX], const T (&Aa)[TB][RY][VX],
                                                int r, unsigned long long mask) {
    static_assert(TB >= 3 && TB <= 8 && VX == 1, "ghost reset: 3..8 levels, one site per lane");
    unsigned long long sv;
#define GR_HEAD "s_and_saveexec_b64 %[sv], %[m]\n\ts_cbranch_execz 1f\n\t"
#define GR_TAIL "1:\n\ts_mov_b64 exec, %[sv]"
    if constexpr (sizeof(T) == 8) {
#define GR_M(d, s) "v_mov_b64 %[" #d "], %[" #s "]\n\t"
        if constexpr (TB == 3) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 4) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 5) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_M(d4, s4) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [d4] "+v"(Bb[4][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [s4] "v"(Aa[3][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 6) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_M(d4, s4)
                                 GR_M(d5, s5) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [d4] "+v"(Bb[4][r][0]),
                               [d5] "+v"(Bb[5][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [s4] "v"(Aa[3][r][0]),
                               [s5] "v"(Aa[4][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 7) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_M(d4, s4)
                                 GR_M(d5, s5) GR_M(d6, s6) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [d4] "+v"(Bb[4][r][0]),
                               [d5] "+v"(Bb[5][r][0]), [d6] "+v"(Bb[6][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [s4] "v"(Aa[3][r][0]),
                               [s5] "v"(Aa[4][r][0]), [s6] "v"(Aa[5][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 8) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_M(d4, s4)
                                 GR_M(d5, s5) GR_M(d6, s6) GR_M(d7, s7) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [d4] "+v"(Bb[4][r][0]),
                               [d5] "+v"(Bb[5][r][0]), [d6] "+v"(Bb[6][r][0]),
                               [d7] "+v"(Bb[7][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [s4] "v"(Aa[3][r][0]),
                               [s5] "v"(Aa[4][r][0]), [s6] "v"(Aa[5][r][0]),
                               [s7] "v"(Aa[6][r][0]), [m] "s"(mask)
                             : "scc");
        }
#undef GR_M
    } else {
#define GR_M(d, s) "v_mov_b32 %[" #d "], %[" #s "]\n\t"
        if constexpr (TB == 3) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 4) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 5) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_M(d4, s4) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [d4] "+v"(Bb[4][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [s4] "v"(Aa[3][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 6) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_M(d4, s4)
                                 GR_M(d5, s5) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [d4] "+v"(Bb[4][r][0]),
                               [d5] "+v"(Bb[5][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [s4] "v"(Aa[3][r][0]),
                               [s5] "v"(Aa[4][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 7) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_M(d4, s4)
                                 GR_M(d5, s5) GR_M(d6, s6) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [d4] "+v"(Bb[4][r][0]),
                               [d5] "+v"(Bb[5][r][0]), [d6] "+v"(Bb[6][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [s4] "v"(Aa[3][r][0]),
                               [s5] "v"(Aa[4][r][0]), [s6] "v"(Aa[5][r][0]), [m] "s"(mask)
                             : "scc");
        } else if constexpr (TB == 8) {
            __asm__ volatile(GR_HEAD GR_M(d1, s1) GR_M(d2, s2) GR_M(d3, s3) GR_M(d4, s4)
                                 GR_M(d5, s5) GR_M(d6, s6) GR_M(d7, s7) GR_TAIL
                             : [d1] "+v"(Bb[1][r][0]), [d2] "+v"(Bb[2][r][0]),
                               [d3] "+v"(Bb[3][r][0]), [d4] "+v"(Bb[4][r][0]),
                               [d5] "+v"(Bb[5][r][0]), [d6] "+v"(Bb[6][r][0]),
                               [d7] "+v"(Bb[7][r][0]), [sv] "=&s"(sv)
                             : [s1] "v"(Aa[0][r][0]), [s2] "v"(Aa[1][r][0]),
                               [s3] "v"(Aa[2][r][0]), [s4] "v"(Aa[3][r][0]),
                               [s5] "v"(Aa[4][r][0]), [s6] "v"(Aa[5][r][0]),
                               [s7] "v"(Aa[6][r][0]), [m] "s"(mask)
                             : "scc");
        }
#undef GR_M
    }
#undef GR_HEAD
#undef GR_TAIL
}

// RB: red-black Gauss-Seidel.  Level tau updates only the sites of colour
// (tau - 1) & 1 (colour = parity of (x-h) + (y-h) + (z-h)) and copies the
// others from level tau-1; axis neighbours have the other colour, so two
// levels are one red-black sweep.  Level tau produces plane s - tau at step
// s, so the updated colour at step s is the same for every level: a site is
// updated at step s iff x + y + s - 3h + 1 is even.
template <typename T, int TB, int VX, int RY, int NW, bool HAS_A, bool HAS_F, bool EDGE,
          bool RB = false>
__device__ __forceinline__ void jacobi_tile(const JacArgs<T> &A, int tx, int ty, int cz,
                                            T (*xch)[TB][NW][2][64 * VX], T *fring) {
    constexpr bool RING = FRing<T, TB, VX, RY, NW, HAS_F>::on;
    // level 1 takes f from registers loaded one step early when the ring is
    // used; otherwise every level loads its own f plane
    constexpr bool FPRE = RING;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int h = A.h;
    // Row stores as unconditional buffer stores (see the store at the end of
    // a step) where one point per lane is stored.
    constexpr bool BUF_STORE = VX == 1;
    // Row-major steady-state steps (step_rows) where they measured faster on
    // MI355X at 512^3: tiles of one site per lane (two per lane were slower),
    // two or more levels (FP32: any number), with a right-hand side only with
    // the f ring and in FP64 at two levels or from five up (per-level f loads,
    // and the FP64 three- and four-level tiles with f, were slower), and not
    // for the plain FP32 depth-4 Jacobi pass.  In edge tiles they reset the ghost sites next
    // to the interior once per step (GHOST_RESET).  From five levels in FP64
    // and six in FP32 (EDGE_ASM) edge tiles load through buffer loads that
    // return 0 for sites outside the array and do the reset in asm without
    // compiler-visible branches; below that, loads from clamped addresses and
    // a branch per reset measured faster (FP64 t=3/4 by 2-3 %, FP32 t=5 by 2 %).
    constexpr bool ROWS = VX == 1 && (TB >= 2 || sizeof(T) == 4) &&
                          (!HAS_F || (RING && (TB >= 5 || TB == 2 || sizeof(T) == 4))) &&
                          !(sizeof(T) == 4 && TB == 4 && !RB && !HAS_F);
    constexpr bool GHOST_RESET = ROWS && EDGE;
    constexpr bool EDGE_ASM = GHOST_RESET && TB >= (sizeof(T) == 8 ? 5 : 6);
    constexpr bool EDGE_BUF_LOAD = EDGE_ASM;
    constexpr bool CLAMPED = GHOST_RESET && !EDGE_ASM;

    // ---- tile geometry (padded coordinates) ----
    const int ox0 = h + tx * A.ow;
    const int ox1 = min(ox0 + A.ow, h + A.nx);
    int xs = ox0 - TB;
    xs -= ((xs % VX) + VX) % VX;  // align the tile start to the vector width
    const int oy0 = h + ty * A.oh;
    const int oy1 = min(oy0 + A.oh, h + A.ny);
    const int ys = oy0 - TB;
    const int z0 = h + cz * A.zc;
    const int z1 = min(z0 + A.zc, h + A.nz);
    int zb = z0 - TB;
    if (zb < h - 1) zb = h - 1;          // never below the ghost plane
    int ze = z1 - 1 + TB;
    bool top_bnd = false;
    if (ze >= h + A.nz) { ze = h + A.nz; top_bnd = true; }  // ghost plane on top

    const int x0 = xs + lane * VX;  // this lane's first x
    const int y0 = ys + w * RY;     // this wave's first row

    // ---- per-thread masks ----
    unsigned ldx = 0, updx = 0, stx = 0, ldy = 0, updy = 0, sty = 0;
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const int x = x0 + v;
        ldx |= (x >= 0 && x < A.nx + 2 * h) ? (1u << v) : 0u;
        updx |= (x >= h && x < h + A.nx) ? (1u << v) : 0u;
        stx |= (x >= ox0 && x < ox1) ? (1u << v) : 0u;
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = y0 + r;
        ldy |= (y >= 0 && y < A.ny + 2 * h) ? (1u << r) : 0u;
        updy |= (y >= h && y < h + A.ny) ? (1u << r) : 0u;
        sty |= (y >= oy0 && y < oy1) ? (1u << r) : 0u;
    }
    // element offset of (row r, x0) within a plane; rows outside the array are
    // never dereferenced (EDGE masks), so clamping them keeps offsets sane.
    // With EDGE_BUF_LOAD a site outside the array gets the offset of the next
    // plane instead, which a buffer load of this plane treats as out of range
    // (it returns 0 without a memory access); sites inside the array (all
    // that load, store or are masked loads' targets) keep their offset.
    // With CLAMPED the x offset is clamped instead, so that an unmasked load
    // stays inside the array.
    int rowoff[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        int y = y0 + r;
        if (EDGE) y = min(max(y, 0), A.ny + 2 * h - 1);
        rowoff[r] = y * (int)A.px + (CLAMPED ? min(max(x0, 0), (int)A.px - 1) : x0);
        if (EDGE_BUF_LOAD && !((ldy >> r & 1u) && (ldx & 1u))) rowoff[r] = (int)A.plane;
    }
    // the ghost column / rows adjacent to the interior (GHOST_RESET): the
    // lanes holding the column, and per wave the rows that are ghost rows
    unsigned gxm = 0, gym = 0;
#pragma unroll
    for (int v = 0; v < VX; ++v) {
        const int x = x0 + v;
        gxm |= (x == h - 1 || x == h + A.nx) ? (1u << v) : 0u;
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = y0 + r;
        gym |= (y == h - 1 || y == h + A.ny) ? (1u << r) : 0u;
    }
    gym = __builtin_amdgcn_readfirstlane(gym);
    const unsigned long long gx_lanes = __builtin_amdgcn_ballot_w64(gxm != 0u);

    auto load_plane = [&](int z, T (&out)[RY][VX]) {
        const T *base = A.src + (int64_t)z * A.plane;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const unsigned ok = (ldy >> r & 1u) ? ldx : 0u;
            load_row<T, VX, EDGE>(base + rowoff[r], ok, out[r]);
        }
    };
    auto load_f = [&](int z, T (&out)[RY][VX]) {
        // f is interior-only: f[((z-h)*ny + (y-h))*nx + (x-h)].  Planes
        // outside the interior (only read by levels that copy there) are
        // clamped to a valid plane.
        const int zc = min(max(z, h), h + A.nz - 1);
        const T *base = A.f + ((int64_t)(zc - h) * A.ny) * A.nx;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const unsigned ok = (updy >> r & 1u) ? updx : 0u;
            const int y = EDGE ? min(max(y0 + r, h), h + A.ny - 1) : y0 + r;
            load_row<T, VX, EDGE>(base + (int64_t)(y - h) * A.nx + (x0 - h), ok, out[r]);
        }
    };

    // Two planes per level live in registers, in arrays P0 and P1 whose roles
    // alternate from step to step.  At the start of step s, "A" holds
    // A[k] = L_k[s-k-1] (newest plane of level k) and "B" holds
    // B[k] = L_k[s-k-2]; the edge rows of every A[k] were exchanged through
    // LDS at the end of the previous step.  Level tau at plane p = s-tau needs
    // A[tau-1] (centre and in-plane neighbours), B[tau-1][site] (z-) and the
    // new plane of level tau-1 at the same site (z+); once read, B[tau-1][site]
    // is dead and is overwritten by that new plane, so after the step the "B"
    // array holds the newest planes and the roles swap -- no register moves.
    T P0[TB][RY][VX];
    T P1[TB][RY][VX];
    T nxt[RY][VX];
    // f of plane s-1 (for level 1 at step s) and of plane s (loaded at step s),
    // alternating like P0/P1
    T F0[FPRE ? RY : 1][VX];
    T F1[FPRE ? RY : 1][VX];
    const int tid = threadIdx.x;
    auto ring_slot = [&](int plane) {
        constexpr int M = TB > 1 ? TB - 1 : 1;
        return ((plane % M) + M) % M;
    };
    auto ring_at = [&](int slot, int r, int v) -> T & {
        return fring[((slot * RY + r) * VX + v) * (NW * 64) + tid];
    };

    auto exchange = [&](int buf, T (&Anew)[TB][RY][VX]) {
        if constexpr (NW > 1) {
#pragma unroll
            for (int k = 0; k < TB; ++k) {
                T *x0 = &xch[buf][k][w][0][lane * VX];
                T *x1 = &xch[buf][k][w][1][lane * VX];
#pragma unroll
                for (int v = 0; v < VX; ++v) x0[v] = Anew[k][0][v], x1[v] = Anew[k][RY - 1][v];
            }
        }
        __syncthreads();
    };

    // prologue: plane zb is known at every level (ghost plane, or a warm-up
    // plane whose levels never reach a stored output)
    load_plane(zb, nxt);
#pragma unroll
    for (int k = 0; k < TB; ++k)
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int v = 0; v < VX; ++v) P0[k][r][v] = nxt[r][v], P1[k][r][v] = nxt[r][v];
    if (zb + 1 <= ze) load_plane(zb + 1, nxt);
    if constexpr (FPRE) load_f(zb, F0);
    int buf = 0;
    exchange(buf, P0);
    const int s_end = z1 - 1 + TB;

    // FULL: steady state, every level produces and the next plane exists
    auto step = [&](int s, T (&Aa)[TB][RY][VX], T (&Bb)[TB][RY][VX],
                    T (&Fc)[FPRE ? RY : 1][VX], T (&Fn)[FPRE ? RY : 1][VX], auto full_c) {
        constexpr bool FULL = decltype(full_c)::value;
        // red-black: parity of the sites this step updates, for (r, v) = (0, 0)
        const int rbp = RB ? ((x0 + y0 + s + 1 - 3 * h) & 1) : 0;
        T Nprev[RY][VX];  // new plane of level tau-1 (level 0: plane s, loaded)
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int v = 0; v < VX; ++v) Nprev[r][v] = nxt[r][v];
        if (FULL || s + 1 <= ze) load_plane(s + 1, nxt);
        if constexpr (FPRE) load_f(s, Fn);  // for level 1 at step s+1

#pragma unroll
        for (int tau = 1; tau <= TB; ++tau) {
            const int p = s - tau;  // plane of level tau produced now
            const int ce = top_bnd ? ze - 1 : ze - tau;
            // Planes outside [zb+1, ce] take the value of the level below:
            // ghost planes keep their Dirichlet value, elsewhere the value is
            // never used.
            const bool inr = FULL || (p >= zb + 1 && p <= ce);
            T Ncur[RY][VX];
            auto update = [&]() {
                // in-plane neighbours of L_{tau-1}[p] = Aa[tau-1]
                T lft[RY], rgt[RY], ytop[VX], ybot[VX];
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    lft[r] = from_lower_lane(Aa[tau - 1][r][VX - 1]);
                    rgt[r] = from_upper_lane(Aa[tau - 1][r][0]);
                }
                if constexpr (NW > 1) {
                    const T *up = &xch[buf][tau - 1][w > 0 ? w - 1 : w][1][lane * VX];
                    const T *dn = &xch[buf][tau - 1][w < NW - 1 ? w + 1 : w][0][lane * VX];
#pragma unroll
                    for (int v = 0; v < VX; ++v) ytop[v] = up[v], ybot[v] = dn[v];
                } else {
#pragma unroll
                    for (int v = 0; v < VX; ++v)
                        ytop[v] = Aa[tau - 1][0][v], ybot[v] = Aa[tau - 1][RY - 1][v];
                }
                T fv[HAS_F ? RY : 1][VX];
                if constexpr (HAS_F) {
                    if (FPRE && tau == 1) {
#pragma unroll
                        for (int r = 0; r < RY; ++r)
#pragma unroll
                            for (int v = 0; v < VX; ++v) fv[r][v] = Fc[FPRE ? r : 0][v];
                    } else if constexpr (RING) {
                        const int sl = ring_slot(p);
#pragma unroll
                        for (int r = 0; r < RY; ++r)
#pragma unroll
                            for (int v = 0; v < VX; ++v) fv[r][v] = ring_at(sl, r, v);
                    } else if (inr) {
                        load_f(p, fv);
                    } else {
#pragma unroll
                        for (int r = 0; r < RY; ++r)
#pragma unroll
                            for (int v = 0; v < VX; ++v) fv[r][v] = T(0);
                    }
                }
#pragma unroll
                for (int r = 0; r < RY; ++r)
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        const T c = Aa[tau - 1][r][v];
                        const T xm = (v > 0) ? Aa[tau - 1][r][v - 1] : lft[r];
                        const T xp = (v < VX - 1) ? Aa[tau - 1][r][v + 1] : rgt[r];
                        const T ym = (r > 0) ? Aa[tau - 1][r - 1][v] : ytop[v];
                        const T yp = (r < RY - 1) ? Aa[tau - 1][r + 1][v] : ybot[v];
                        const T sum =
                            ((((xm + xp) + ym) + yp) + Bb[tau - 1][r][v]) + Nprev[r][v];
                        T val;
                        if constexpr (HAS_A)
                            val = (A.a * c) + (A.b * sum);
                        else
                            val = A.b * sum;
                        if constexpr (HAS_F) val = val + (A.g * fv[r][v]);
                        if constexpr (RB) val = ((rbp + r + v) & 1) ? c : val;
                        if constexpr (EDGE) {
                            const bool up = (updy >> r & 1u) && (updx >> v & 1u);
                            val = up ? val : c;
                        }
                        Ncur[r][v] = val;
                        Bb[tau - 1][r][v] = Nprev[r][v];
                    }
            };
            auto copy_below = [&]() {
#pragma unroll
                for (int r = 0; r < RY; ++r)
#pragma unroll
                    for (int v = 0; v < VX; ++v) {
                        Ncur[r][v] = Aa[tau - 1][r][v];
                        Bb[tau - 1][r][v] = Nprev[r][v];
                    }
            };
            if constexpr (TB >= 2) {
                // The update runs on every step (it reads only registers and
                // LDS) and the few fill/drain steps overwrite it afterwards: the
                // common path then carries no register copies.  (Measured: this
                // is faster for TB >= 2 and slower for TB = 1.)
                update();
                if (__builtin_expect(!inr, 0)) copy_below();
            } else {
                if (inr)
                    update();
                else
                    copy_below();
            }
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int v = 0; v < VX; ++v) Nprev[r][v] = Ncur[r][v];
        }
        // plane s-1 of f joins the ring, in the slot of plane s-TB (read by
        // level TB above: each thread only touches its own entries, in order)
        if constexpr (RING) {
            const int sl = ring_slot(s - 1);
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int v = 0; v < VX; ++v) ring_at(sl, r, v) = Fc[r][v];
        }
        // store level TB of plane s-TB
        const int p = s - TB;
        if constexpr (BUF_STORE) {
            // One buffer store per row, issued on every step: lanes that must
            // not write get an offset past the plane, which the buffer unit
            // drops.  Stores issued unconditionally let the wait for the next
            // plane's loads (the memory counter retires in issue order) leave
            // this step's stores in flight; behind a branch the count would
            // have to assume no store was issued and wait for them as well.
            const bool pin = p >= z0 && p < z1;
            const int nrec = (int)(A.plane * (int64_t)sizeof(T));
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                A.dst + (int64_t)(pin ? p : z0) * A.plane, 0, nrec, 0x00020000);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const bool ok = pin && (sty >> r & 1u) && (stx & 1u);
                const int off = ok ? rowoff[r] * (int)sizeof(T) : nrec;
                if constexpr (sizeof(T) == 8)
                    __builtin_amdgcn_raw_buffer_store_b64(
                        __builtin_bit_cast(U32x2, Nprev[r][0]), rs, off, 0, 0);
                else
                    __builtin_amdgcn_raw_buffer_store_b32(
                        __builtin_bit_cast(unsigned, Nprev[r][0]), rs, off, 0, 0);
            }
        } else if (p >= z0 && p < z1) {
            T *base = A.dst + (int64_t)p * A.plane;
#pragma unroll
            for (int r = 0; r < RY; ++r)
                if (sty >> r & 1u) store_row<T, VX>(base + rowoff[r], stx, Nprev[r]);
        }
        buf ^= 1;
        exchange(buf, Bb);
    };

    // Row-major steady-state step (ROWS): every level produces an
    // in-range plane and the next plane exists.  For one row at a time it
    // first forms, for every level, the partial sum up to the z- term --
    // these read only planes of the previous step -- and then completes the
    // levels bottom up: level tau adds the new plane of level tau-1 (z+) and
    // writes its own new plane straight into the register of the z- plane it
    // has just consumed.  The arithmetic and its order are those of `step`;
    // what changes is that the plane rotation needs no register copies (the
    // level-major step keeps a new plane in a temporary until the level
    // above has read the plane it replaces).
    //
    // Edge tiles: within a step a site reads other sites only in planes of
    // the previous step (the new plane of the level below is read at the
    // same site), so the ghost sites next to the interior -- the only ones
    // whose values reach an interior site -- are reset to the level below
    // once, at the end of the step, instead of masking every update.  Sites
    // farther out (loaded as 0 by out-of-range buffer loads, or from clamped
    // addresses) hold values nothing stored depends on.
    auto step_rows = [&](int s, T (&Aa)[TB][RY][VX], T (&Bb)[TB][RY][VX],
                         T (&Fc)[FPRE ? RY : 1][VX], T (&Fn)[FPRE ? RY : 1][VX]) {
        const int rbp = RB ? ((x0 + y0 + s + 1 - 3 * h) & 1) : 0;
        // plane s of level 0 (loaded one step early); plane s+1 is loaded now
        T in0[RY][VX];
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int v = 0; v < VX; ++v) in0[r][v] = nxt[r][v];
        if constexpr (EDGE_BUF_LOAD) {
            const __amdgpu_buffer_rsrc_t rl = __builtin_amdgcn_make_buffer_rsrc(
                const_cast<T *>(A.src) + (int64_t)(s + 1) * A.plane, 0,
                (int)(A.plane * (int64_t)sizeof(T)), 0x00020000);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                const int off = rowoff[r] * (int)sizeof(T);
                if constexpr (sizeof(T) == 8)
                    nxt[r][0] = __builtin_bit_cast(
                        T, __builtin_amdgcn_raw_buffer_load_b64(rl, off, 0, 0));
                else
                    nxt[r][0] = __builtin_bit_cast(
                        T, __builtin_amdgcn_raw_buffer_load_b32(rl, off, 0, 0));
            }
        } else if constexpr (CLAMPED) {
            const T *base = A.src + (int64_t)(s + 1) * A.plane;
#pragma unroll
            for (int r = 0; r < RY; ++r) nxt[r][0] = base[rowoff[r]];
        } else {
            load_plane(s + 1, nxt);
        }
        if constexpr (FPRE) load_f(s, Fn);  // for level 1 at step s+1
        const int p_out = s - TB;
        const bool pin = p_out >= z0 && p_out < z1;
        const int nrec = (int)(A.plane * (int64_t)sizeof(T));
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            A.dst + (int64_t)(pin ? p_out : z0) * A.plane, 0, nrec, 0x00020000);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            T part[TB][VX];
#pragma unroll
            for (int tau = 1; tau <= TB; ++tau) {
                const T lft = from_lower_lane(Aa[tau - 1][r][VX - 1]);
                const T rgt = from_upper_lane(Aa[tau - 1][r][0]);
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const T xm = (v > 0) ? Aa[tau - 1][r][v - 1] : lft;
                    const T xp = (v < VX - 1) ? Aa[tau - 1][r][v + 1] : rgt;
                    T ym, yp;
                    if (r > 0) {
                        ym = Aa[tau - 1][r - 1][v];
                    } else if constexpr (NW > 1) {
                        ym = xch[buf][tau - 1][w > 0 ? w - 1 : w][1][lane * VX + v];
                    } else {
                        ym = Aa[tau - 1][0][v];
                    }
                    if (r < RY - 1) {
                        yp = Aa[tau - 1][r + 1][v];
                    } else if constexpr (NW > 1) {
                        yp = xch[buf][tau - 1][w < NW - 1 ? w + 1 : w][0][lane * VX + v];
                    } else {
                        yp = Aa[tau - 1][RY - 1][v];
                    }
                    part[tau - 1][v] = (((xm + xp) + ym) + yp) + Bb[tau - 1][r][v];
                }
            }
#pragma unroll
            for (int v = 0; v < VX; ++v) Bb[0][r][v] = in0[r][v];
            T outv[VX];
#pragma unroll
            for (int tau = 1; tau <= TB; ++tau) {
                T fv[VX];
                if constexpr (HAS_F) {
                    if (FPRE && tau == 1) {
#pragma unroll
                        for (int v = 0; v < VX; ++v) fv[v] = Fc[FPRE ? r : 0][v];
                    } else if constexpr (RING) {
                        const int sl = ring_slot(s - tau);
#pragma unroll
                        for (int v = 0; v < VX; ++v) fv[v] = ring_at(sl, r, v);
                    } else {
                        const int y = EDGE ? min(max(y0 + r, h), h + A.ny - 1) : y0 + r;
                        const unsigned ok = (updy >> r & 1u) ? updx : 0u;
                        load_row<T, VX, EDGE>(
                            A.f + ((int64_t)(s - tau - h) * A.ny + (y - h)) * A.nx + (x0 - h), ok,
                            fv);
                    }
                }
#pragma unroll
                for (int v = 0; v < VX; ++v) {
                    const T c = Aa[tau - 1][r][v];
                    const T sum = part[tau - 1][v] + Bb[tau - 1][r][v];
                    T val;
                    if constexpr (HAS_A)
                        val = (A.a * c) + (A.b * sum);
                    else
                        val = A.b * sum;
                    if constexpr (HAS_F) val = val + (A.g * fv[v]);
                    if constexpr (RB) val = ((rbp + r + v) & 1) ? c : val;
                    if constexpr (EDGE && !GHOST_RESET) {
                        const bool up = (updy >> r & 1u) && (updx >> v & 1u);
                        val = up ? val : c;
                    }
                    if (tau < TB)
                        Bb[tau < TB ? tau : 0][r][v] = val;
                    else
                        outv[v] = val;
                }
            }
            // store row r of level TB (plane s-TB), as in `step`
            if constexpr (BUF_STORE) {
                const bool ok = pin && (sty >> r & 1u) && (stx & 1u);
                const int off = ok ? rowoff[r] * (int)sizeof(T) : nrec;
                if constexpr (sizeof(T) == 8)
                    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U32x2, outv[0]), rs,
                                                          off, 0, 0);
                else
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, outv[0]),
                                                          rs, off, 0, 0);
            } else if (pin && (sty >> r & 1u)) {
                store_row<T, VX>(A.dst + (int64_t)p_out * A.plane + rowoff[r], stx, outv);
            }
            // keep the scheduler from interleaving rows: the rows' partial
            // sums would then be live together and spill
            __builtin_amdgcn_sched_barrier(0);
        }
        // levels 1..TB-1 keep their new plane (level TB's is only stored)
        if constexpr (EDGE_ASM) {
#pragma unroll
            for (int r = 0; r < RY; ++r)
                ghost_reset_row<T, TB, RY, VX>(Bb, Aa, r, (gym >> r & 1u) ? ~0ull : gx_lanes);
        } else if constexpr (GHOST_RESET) {
            if (gxm) {
                __asm__ volatile("" ::: "memory");  // keep this a masked region
#pragma unroll
                for (int k = 1; k < TB; ++k)
#pragma unroll
                    for (int r = 0; r < RY; ++r)
                        Bb[k][r][0] = Aa[k - 1][r][0];
            }
            if (gym) {
#pragma unroll
                for (int r = 0; r < RY; ++r)
                    if (gym >> r & 1u) {
                        __asm__ volatile("" ::: "memory");
#pragma unroll
                        for (int k = 1; k < TB; ++k) Bb[k][r][0] = Aa[k - 1][r][0];
                    }
            }
        }
        if constexpr (RING) {
            const int sl = ring_slot(s - 1);
#pragma unroll
            for (int r = 0; r < RY; ++r)
#pragma unroll
                for (int v = 0; v < VX; ++v) ring_at(sl, r, v) = Fc[r][v];
        }
        buf ^= 1;
        exchange(buf, Bb);
    };

    using Part = std::integral_constant<bool, false>;
    // Drain the prologue's loads here (vmcnt(0); expcnt and lgkmcnt left at
    // their maxima): otherwise the loop header has to assume them pending and
    // waits for every outstanding store on each iteration.
    __builtin_amdgcn_s_waitcnt(0x0F70);
    int s = zb + 1;
    // last step that may load the next plane: below the top ghost plane, or
    // anywhere in a chunk whose warm-up end lies inside the grid (plane ze+1
    // exists there)
    const int last_full = top_bnd ? ze - 1 : s_end;
    if constexpr (ROWS) {
        // Three loops over pairs of steps (the planes alternate between P0
        // and P1, so every loop starts with P0 holding the newest planes):
        // checked level-major steps while the pipeline fills (some level's
        // plane still lies below zb+1), row-major steady-state steps while
        // every level is in range and the next plane exists, checked steps
        // for the rest (the top ghost plane).  Chunks too short for a
        // steady pair use checked steps throughout.  Each loop keeps to one
        // kind of step: a loop choosing between the two made the register
        // allocator spill.
        const int full_lo = zb + 1 + TB;
        if (full_lo + 1 <= last_full) {
            for (; s < full_lo; s += 2) {
                step(s, P0, P1, F0, F1, Part{});
                step(s + 1, P1, P0, F1, F0, Part{});
            }
            for (; s + 1 <= last_full; s += 2) {
                step_rows(s, P0, P1, F0, F1);
                step_rows(s + 1, P1, P0, F1, F0);
            }
        }
        for (; s + 1 <= s_end; s += 2) {
            step(s, P0, P1, F0, F1, Part{});
            step(s + 1, P1, P0, F1, F0, Part{});
        }
        if (s <= s_end) step(s, P0, P1, F0, F1, Part{});
    } else {
        for (; s + 1 <= s_end; s += 2) {
            step(s, P0, P1, F0, F1, Part{});
            step(s + 1, P1, P0, F1, F0, Part{});
        }
        if (s <= s_end) step(s, P0, P1, F0, F1, Part{});
    }
}

// A tile takes the unmasked path when its whole loaded footprint (the stored
// tile plus TB sites on every side, x start aligned to the vector width) lies
// inside the interior.  Shared by the kernels and the host-side tile count.
template <int TB, int VX, int RY, int NW>
__host__ __device__ __forceinline__ bool tile_interior(int h, int nx, int ny, int ow, int oh,
                                                       int tx, int ty) {
    int xs = h + tx * ow - TB;
    xs -= ((xs % VX) + VX) % VX;
    const int ys = h + ty * oh - TB;
    return xs >= h && xs + 64 * VX <= h + nx && ys >= h && ys + NW * RY <= h + ny;
}

template <typename T, int TB, int VX, int RY, int NW, bool HAS_A, bool HAS_F, bool RB = false>
__global__ void __launch_bounds__(NW * 64) jacobi_pass_kernel(JacArgs<T> A) {
    __shared__ T xch[2][TB][NW][2][64 * VX];
    __shared__ T fring[FRing<T, TB, VX, RY, NW, HAS_F>::alloc];
    // The dispatcher places consecutive workgroup ids round-robin on the 8
    // XCDs; give each XCD a contiguous range of tiles so that neighbouring
    // tiles (which re-read each other's overlap) share an L2.
    const int G = gridDim.x;
    const int per = G >> 3;
    const int bid = blockIdx.x;
    const int l = (bid & 7) * per + (bid >> 3);
    if (l >= A.ntiles) return;
    const int tpc = A.tiles_x * A.tiles_y;
    const int cz = l / tpc;
    const int rem = l - cz * tpc;
    const int ty = rem / A.tiles_x;
    const int tx = rem - ty * A.tiles_x;

    if (tile_interior<TB, VX, RY, NW>(A.h, A.nx, A.ny, A.ow, A.oh, tx, ty))
        jacobi_tile<T, TB, VX, RY, NW, HAS_A, HAS_F, false, RB>(A, tx, ty, cz, xch, fring);
    else
        jacobi_tile<T, TB, VX, RY, NW, HAS_A, HAS_F, true, RB>(A, tx, ty, cz, xch, fring);
}

// Batched pass: one launch advances several independent grids (jobs of the
// job service) by one fused pass each.  jobs[j].wg_begin is the prefix sum of
// the workgroups of the jobs before j; a workgroup finds its job by binary
// search and then runs exactly the single-grid tile code, so a job's result
// does not depend on which other jobs share the launch.
template <typename T>
struct JacJob {
    JacArgs<T> a;
    int wg_begin;
    int pad_[3];
};

template <typename T, int TB, int VX, int RY, int NW, bool HAS_A, bool HAS_F>
__global__ void __launch_bounds__(NW * 64)
    jacobi_batch_kernel(const JacJob<T> *__restrict__ jobs, int njobs, int total) {
    __shared__ T xch[2][TB][NW][2][64 * VX];
    __shared__ T fring[FRing<T, TB, VX, RY, NW, HAS_F>::alloc];
    const int G = gridDim.x;
    const int per = G >> 3;
    const int bid = blockIdx.x;
    const int l = (bid & 7) * per + (bid >> 3);
    if (l >= total) return;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].wg_begin <= l) lo = mid; else hi = mid - 1;
    }
    const JacArgs<T> A = jobs[lo].a;
    const int li = l - jobs[lo].wg_begin;
    const int tpc = A.tiles_x * A.tiles_y;
    const int cz = li / tpc;
    const int rem = li - cz * tpc;
    const int ty = rem / A.tiles_x;
    const int tx = rem - ty * A.tiles_x;
    if (tile_interior<TB, VX, RY, NW>(A.h, A.nx, A.ny, A.ow, A.oh, tx, ty))
        jacobi_tile<T, TB, VX, RY, NW, HAS_A, HAS_F, false>(A, tx, ty, cz, xch, fring);
    else
        jacobi_tile<T, TB, VX, RY, NW, HAS_A, HAS_F, true>(A, tx, ty, cz, xch, fring);
}

// Tile configurations (VX, RY, NW), chosen by measurement on MI355X among
// shapes that fit the register file: per thread about (2*TB + 3) * RY * VX
// values stay live, which must fit 256 VGPRs (two waves per SIMD), while the
// tile must be large against the 2*TB overlap on each side.
template <typename T, int TB>
struct CfgBase;
template <> struct CfgBase<double, 1> { static constexpr int VX = 2, RY = 4, NW = 8; };
template <> struct CfgBase<double, 2> { static constexpr int VX = 2, RY = 4, NW = 8; };
template <> struct CfgBase<double, 3> { static constexpr int VX = 1, RY = 10, NW = 8; };
template <> struct CfgBase<double, 4> { static constexpr int VX = 1, RY = 9, NW = 8; };
template <> struct CfgBase<double, 5> { static constexpr int VX = 1, RY = 7, NW = 8; };
template <> struct CfgBase<double, 6> { static constexpr int VX = 1, RY = 6, NW = 8; };
template <> struct CfgBase<double, 7> { static constexpr int VX = 1, RY = 5, NW = 8; };
template <> struct CfgBase<double, 8> { static constexpr int VX = 1, RY = 5, NW = 8; };
template <> struct CfgBase<float, 1> { static constexpr int VX = 1, RY = 16, NW = 8; };
template <> struct CfgBase<float, 2> { static constexpr int VX = 1, RY = 16, NW = 8; };
template <> struct CfgBase<float, 3> { static constexpr int VX = 1, RY = 12, NW = 8; };
template <> struct CfgBase<float, 4> { static constexpr int VX = 1, RY = 12, NW = 8; };
template <> struct CfgBase<float, 5> { static constexpr int VX = 1, RY = 12, NW = 8; };
template <> struct CfgBase<float, 6> { static constexpr int VX = 1, RY = 8, NW = 8; };
template <> struct CfgBase<float, 7> { static constexpr int VX = 1, RY = 9, NW = 8; };
template <> struct CfgBase<float, 8> { static constexpr int VX = 1, RY = 8, NW = 8; };
// With a right-hand side the prefetched f planes add register pressure and
// the f ring needs LDS next to the exchange buffer: some shapes are shorter
// (FP32 t=8 also so that its ring fits; FP64 t=8 has no room for the ring
// and loads f per level).
template <typename T, int TB, bool HAS_F>
struct Cfg : CfgBase<T, TB> {};
template <> struct Cfg<double, 2, true> { static constexpr int VX = 1, RY = 8, NW = 8; };
template <> struct Cfg<double, 3, true> { static constexpr int VX = 1, RY = 6, NW = 8; };
template <> struct Cfg<double, 4, true> { static constexpr int VX = 1, RY = 7, NW = 8; };
template <> struct Cfg<double, 5, true> { static constexpr int VX = 1, RY = 5, NW = 8; };
template <> struct Cfg<double, 6, true> { static constexpr int VX = 1, RY = 5, NW = 8; };
template <> struct Cfg<double, 7, true> { static constexpr int VX = 1, RY = 4, NW = 8; };
template <> struct Cfg<double, 8, true> { static constexpr int VX = 1, RY = 4, NW = 8; };
template <> struct Cfg<float, 3, true> { static constexpr int VX = 1, RY = 8, NW = 8; };
template <> struct Cfg<float, 4, true> { static constexpr int VX = 1, RY = 8, NW = 8; };
template <> struct Cfg<float, 5, true> { static constexpr int VX = 1, RY = 8, NW = 8; };
template <> struct Cfg<float, 6, true> { static constexpr int VX = 1, RY = 7, NW = 8; };
template <> struct Cfg<float, 7, true> { static constexpr int VX = 1, RY = 8, NW = 8; };
template <> struct Cfg<float, 8, true> { static constexpr int VX = 1, RY = 6, NW = 8; };

template <typename T, int TB, bool HAS_F = false>
JacTileCfg cfg_of() {
    return JacTileCfg{TB, Cfg<T, TB, HAS_F>::VX, Cfg<T, TB, HAS_F>::RY, Cfg<T, TB, HAS_F>::NW};
}

// Number of z-chunks.  Every chunk re-computes TB warm-up planes (and some
// fill/drain steps), while the grid runs in rounds of `resident` workgroups:
// pick the count that minimises rounds * (planes per chunk + fill).
int choose_chunks(const JacTileCfg &c, const Geom &g, int tiles_xy, int resident) {
    if (resident < 1) resident = 256;
    int best = 1;
    double best_cost = 1e300;
    const int maxch = g.nz / 8 > 1 ? g.nz / 8 : 1;
    for (int nch = 1; nch <= maxch; ++nch) {
        const int zc = (g.nz + nch - 1) / nch;
        const long wgs = (long)tiles_xy * nch;
        const long rounds = (wgs + resident - 1) / resident;
        const double cost = (double)rounds * (zc + c.tb + 1);
        if (cost < best_cost - 1e-9) {
            best_cost = cost;
            best = nch;
        }
    }
    return best;
}

template <typename T, int TB, bool HAS_A, bool HAS_F, bool RB = false>
int resident_wgs(bool batch) {
    using C = Cfg<T, TB, HAS_F>;
    // Workgroups of this kernel per CU and CUs per device, cached on first use
    // (concurrent first calls store the same values).
    static std::atomic<int> per_cu_cached[2];
    static std::atomic<int> ncu_cached[64];
    std::atomic<int> &pc = per_cu_cached[batch ? 1 : 0];
    int per_cu = pc.load(std::memory_order_relaxed);
    if (per_cu == 0) {
        const void *kfn =
            batch ? reinterpret_cast<const void *>(
                        jacobi_batch_kernel<T, TB, C::VX, C::RY, C::NW, HAS_A, HAS_F>)
                  : reinterpret_cast<const void *>(
                        jacobi_pass_kernel<T, TB, C::VX, C::RY, C::NW, HAS_A, HAS_F, RB>);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, C::NW * 64, 0) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        pc.store(per_cu, std::memory_order_relaxed);
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return per_cu * 256;
    int ncu = ncu_cached[dev].load(std::memory_order_relaxed);
    if (ncu == 0) {
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess || ncu < 1)
            ncu = 256;
        ncu_cached[dev].store(ncu, std::memory_order_relaxed);
    }
    return per_cu * ncu;
}

template <typename T, int TB, bool HAS_F>
JacArgs<T> make_args(const Geom &g, const void *src, void *dst, const void *f, double a,
                     double b, double gw, int zc, int resident) {
    const JacTileCfg c = cfg_of<T, TB, HAS_F>();
    JacArgs<T> A;
    A.src = static_cast<const T *>(src);
    A.dst = static_cast<T *>(dst);
    A.f = static_cast<const T *>(f);
    A.px = g.px;
    A.plane = g.plane();
    A.nx = g.nx; A.ny = g.ny; A.nz = g.nz; A.h = g.h;
    A.a = (T)a; A.b = (T)b; A.g = (T)gw;
    A.ow = c.ow();
    A.oh = c.oh();
    A.tiles_x = (g.nx + A.ow - 1) / A.ow;
    A.tiles_y = (g.ny + A.oh - 1) / A.oh;
    const int tiles_xy = A.tiles_x * A.tiles_y;
    if (zc <= 0) {
        const int nch = choose_chunks(c, g, tiles_xy, resident);
        zc = (g.nz + nch - 1) / nch;
    }
    A.zc = zc;
    A.nchunks = (g.nz + zc - 1) / zc;
    A.ntiles = tiles_xy * A.nchunks;
    return A;
}

template <typename T, int TB, bool HAS_A, bool HAS_F, bool RB = false>
hipError_t launch_t(const Geom &g, const void *src, void *dst, const void *f, double a, double b,
                    double gw, int zc, hipStream_t s) {
    using C = Cfg<T, TB, HAS_F>;
    const JacArgs<T> A = make_args<T, TB, HAS_F>(g, src, dst, f, a, b, gw, zc,
                                          resident_wgs<T, TB, HAS_A, HAS_F, RB>(false));
    const int grid = ((A.ntiles + 7) / 8) * 8;
    hipLaunchKernelGGL((jacobi_pass_kernel<T, TB, C::VX, C::RY, C::NW, HAS_A, HAS_F, RB>),
                       dim3(grid), dim3(C::NW * 64), 0, s, A);
    return hipGetLastError();
}

template <typename T, int TB, bool HAS_A, bool HAS_F>
hipError_t launch_batch_t(const std::vector<JacBatchItem> &items, void *table_dev,
                          std::vector<unsigned char> &host_buf, hipStream_t s) {
    using C = Cfg<T, TB, HAS_F>;
    const int resident = resident_wgs<T, TB, HAS_A, HAS_F>(true);
    host_buf.resize(items.size() * sizeof(JacJob<T>));
    JacJob<T> *jobs = reinterpret_cast<JacJob<T> *>(host_buf.data());
    int total = 0;
    for (size_t j = 0; j < items.size(); ++j) {
        const JacBatchItem &it = items[j];
        jobs[j].a =
            make_args<T, TB, HAS_F>(it.g, it.src, it.dst, it.f, it.a, it.b, it.gw, 0, resident);
        jobs[j].wg_begin = total;
        total += jobs[j].a.ntiles;
    }
    hipError_t e = hipMemcpyAsync(table_dev, jobs, items.size() * sizeof(JacJob<T>),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    const int grid = ((total + 7) / 8) * 8;
    hipLaunchKernelGGL((jacobi_batch_kernel<T, TB, C::VX, C::RY, C::NW, HAS_A, HAS_F>),
                       dim3(grid), dim3(C::NW * 64), 0, s,
                       static_cast<const JacJob<T> *>(table_dev), (int)items.size(), total);
    return hipGetLastError();
}

template <typename T, int TB>
hipError_t launch_batch_tb(bool ha, bool hf, const std::vector<JacBatchItem> &items,
                           void *table_dev, std::vector<unsigned char> &hb, hipStream_t s) {
    if (ha && hf) return launch_batch_t<T, TB, true, true>(items, table_dev, hb, s);
    if (ha) return launch_batch_t<T, TB, true, false>(items, table_dev, hb, s);
    if (hf) return launch_batch_t<T, TB, false, true>(items, table_dev, hb, s);
    return launch_batch_t<T, TB, false, false>(items, table_dev, hb, s);
}

template <typename T, int TB, bool RB = false>
hipError_t launch_tb(const Geom &g, const void *src, void *dst, const void *f, double a,
                     double b, double gw, int zc, hipStream_t s) {
    const bool ha = (a != 0.0), hf = (f != nullptr);
    if (ha && hf) return launch_t<T, TB, true, true, RB>(g, src, dst, f, a, b, gw, zc, s);
    if (ha) return launch_t<T, TB, true, false, RB>(g, src, dst, f, a, b, gw, zc, s);
    if (hf) return launch_t<T, TB, false, true, RB>(g, src, dst, f, a, b, gw, zc, s);
    return launch_t<T, TB, false, false, RB>(g, src, dst, f, a, b, gw, zc, s);
}

}  // namespace

template <int TB>
JacTileCfg JacobiLevels<TB>::cfg(bool fp32, bool has_f) {
    if (has_f) return fp32 ? cfg_of<float, TB, true>() : cfg_of<double, TB, true>();
    return fp32 ? cfg_of<float, TB>() : cfg_of<double, TB>();
}

template <typename T, int TB, bool HAS_F>
void count_tiles(const Geom &g, int *tiles, int *interior) {
    using C = Cfg<T, TB, HAS_F>;
    const JacTileCfg c = cfg_of<T, TB, HAS_F>();
    const int ow = c.ow(), oh = c.oh();
    const int tx = (g.nx + ow - 1) / ow, ty = (g.ny + oh - 1) / oh;
    int in = 0;
    for (int y = 0; y < ty; ++y)
        for (int x = 0; x < tx; ++x)
            in += tile_interior<TB, C::VX, C::RY, C::NW>(g.h, g.nx, g.ny, ow, oh, x, y) ? 1 : 0;
    *tiles = tx * ty;
    *interior = in;
}

template <int TB>
void JacobiLevels<TB>::tiles(bool fp32, bool has_f, const Geom &g, int *tiles, int *interior) {
    if (fp32)
        has_f ? count_tiles<float, TB, true>(g, tiles, interior)
              : count_tiles<float, TB, false>(g, tiles, interior);
    else
        has_f ? count_tiles<double, TB, true>(g, tiles, interior)
              : count_tiles<double, TB, false>(g, tiles, interior);
}

template <int TB>
hipError_t JacobiLevels<TB>::pass(bool fp32, const Geom &g, const void *src, void *dst,
                                  const void *f, double a, double b, double gw, int zc,
                                  hipStream_t s) {
    return fp32 ? launch_tb<float, TB>(g, src, dst, f, a, b, gw, zc, s)
                : launch_tb<double, TB>(g, src, dst, f, a, b, gw, zc, s);
}

template <int TB>
hipError_t JacobiLevels<TB>::rb_pass(bool fp32, const Geom &g, const void *src, void *dst,
                                     const void *f, double a, double b, double gw,
                                     hipStream_t s) {
    if constexpr (TB % 2 != 0) {
        return hipErrorInvalidValue;  // a red-black sweep is two levels
    } else {
        return fp32 ? launch_tb<float, TB, true>(g, src, dst, f, a, b, gw, 0, s)
                    : launch_tb<double, TB, true>(g, src, dst, f, a, b, gw, 0, s);
    }
}

template <int TB>
hipError_t JacobiLevels<TB>::batch(bool fp32, bool has_a, bool has_f,
                                   const std::vector<JacBatchItem> &items, void *table_dev,
                                   std::vector<unsigned char> &host_buf, hipStream_t s) {
    return fp32 ? launch_batch_tb<float, TB>(has_a, has_f, items, table_dev, host_buf, s)
                : launch_batch_tb<double, TB>(has_a, has_f, items, table_dev, host_buf, s);
}

template <int TB>
size_t JacobiLevels<TB>::table_bytes(int njobs) {
    return (size_t)njobs * (sizeof(JacJob<double>) > sizeof(JacJob<float>) ? sizeof(JacJob<double>)
                                                                           : sizeof(JacJob<float>));
}

}  // namespace stk
