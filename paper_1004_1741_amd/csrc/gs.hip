// gs.hip -- in-place lexicographic Gauss-Seidel as a pipelined wavefront.
//
// Method (Sec. 3 Gauss-Seidel loop nest; Sec. 3 pipeline-parallel scheme and
// Sec. 4 temporal wavefront GS).  A site's update reads fresh x-, y-, z-
// values of the current sweep and old x+, y+, z+ values of the previous one.
// Because the 7-point stencil only couples axis neighbours, the result only
// depends on that fresh/old split, so any schedule that runs site (i,j,k) of
// sweep tau after (i-1,j,k), (i,j-1,k), (i,j,k-1) of sweep tau and after
// (i+1,j,k), (i,j+1,k), (i,j,k+1) of sweep tau-1 reproduces the sequential
// loop bit for bit.  The paper keeps the order by giving each thread of a
// pipeline a sub-block, shifted in time; here:
//
//   * the (j,k) cross-section is cut into bundles of 8x8 x-lines; one wave
//     owns a bundle for one sweep (a work item) and marches along x.  Lane
//     (jj,kk) handles line (j0+jj, k0+kk) and at step T updates position
//     i = T - jj - kk: its fresh y-/z- neighbours were written by lanes
//     (jj-1,kk)/(jj,kk-1) one step earlier, its old y+/z+ neighbours are not
//     yet overwritten by (jj+1,kk)/(jj,kk+1);
//   * the bundle's lines and the four neighbour lines around it are staged in
//     an LDS ring of 32 x positions, loaded and stored in coalesced chunks of
//     8 positions.  Chunk boundaries follow each line's own alignment (chunk c
//     of a line covers positions [8c - s, 8c + 8 - s), s = the element offset
//     of position 0 past an 8-element boundary), so a chunk is one aligned
//     64-byte (FP64) or 32-byte (FP32) segment instead of straddling two:
//     partial-segment writes cost 1.5x the stored bytes at the memory side;
//   * items (tau, J, K) are handed out by an atomic ticket in order of
//     2*tau + J + K, a topological order of their dependencies, so a wave only
//     ever waits on items already held by running waves (no deadlock, no
//     co-residency requirement).  Instead of barriers, a wave publishes a
//     progress counter (chunks stored) per (sweep, bundle) after storing each
//     chunk and polls its neighbours' counters before loading one (grid
//     data and counters are device-scope relaxed atomics, coherent across
//     XCDs; a chunk is published only after its stores have completed).
//     Counters are per sweep because several sweeps of one bundle are in
//     flight at once;
//   * all sweeps of a launch are in flight at once: there is no launch
//     boundary between sweeps, only the counters order sweep tau+1 of a
//     bundle after sweep tau of it and of its neighbours.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"

#pragma clang fp contract(off)

namespace stk {
namespace {

constexpr int GS_C = 8;       // positions per load/store chunk
constexpr int GS_RING = 32;   // ring positions per staged line (4 chunks)
constexpr int GS_SLOTS = 100; // 10 x 10 staged lines (corners unused)
constexpr int GS_SLOT0 = 1;   // first slot held in LDS (slot 0 is an unused corner)

// LDS layout of the ring, per element type.  The ring holds slots 1..98 only
// (slots 0 and 99 are unused corners) and the last one needs no stride
// padding: 97 * S + 32 values.  The LDS footprint of a workgroup (one wave)
// sets how many fit a CU.  FP64 is sensitive to that: S <= 34 keeps six
// workgroups in the 160 KB of a CU (S = 41 allowed five: 19.2 ms against
// 16.4 ms for 384^3 x 50).  Within that limit S = 34 spreads a wave's ring
// reads best: lane (jj, kk) reads value (10 kk + jj + 10) S - jj - kk + const,
// so with S = 33 the jj term vanishes modulo the 32 bank pairs and eight lanes
// share a bank pair; with S = 34 four do.  FP32 is limited by registers to
// eight waves per CU either way and keeps S = 41 (one lane per bank; 10.1 ms
// against 10.2 ms).  The right-hand-side ring holds the bundle's 64 own lines
// only, slot jj * 8 + kk.
template <typename T>
struct GsLds {
    static constexpr int S = sizeof(T) == 8 ? 34 : 41;
    static constexpr int RING_LEN = (GS_SLOTS - 2 - GS_SLOT0) * S + GS_RING;
    static constexpr int FRING_LEN = 63 * S + GS_RING;
    static_assert(S >= GS_RING, "a staged line needs GS_RING positions");
};

template <typename T>
struct GsJob {
    T *u;
    const T *f;
    int64_t px, plane;
    int nx, ny, nz, h;
    T a, b, g;
    int nj, nk;          // bundles in y and z
    int ncs;             // store chunks per line (positions < nx for any shift)
    int ncl;             // load chunks per line (up to the x+ ghost, any shift)
    int nb;              // step blocks
    uint32_t *progress;  // [sweep][bundle]: chunks stored so far
};

template <typename T>
struct GsArgs {
    GsJob<T> job;
    uint32_t nitems;
    const uint32_t *items;   // (tau << 20) | (J << 10) | K, topologically ordered
    uint32_t *ticket;
};

// Batched launch: items of several jobs merged in key order; each item is
// (job << 48) | (tau << 32) | (J << 16) | K.
template <typename T>
struct GsBatchArgs {
    const GsJob<T> *jobs;
    uint32_t nitems;
    const uint64_t *items;
    uint32_t *ticket;
};

// Bundle data crosses workgroups that may sit on different XCDs, whose L2
// caches are not coherent with each other.  Every access to the grid inside
// this kernel is a device-scope (agent) relaxed atomic: such loads and stores
// are coherent across XCDs by themselves, so publishing a chunk only needs the
// stores to have completed before the progress counter is written, instead of
// the whole-L2 write-back / invalidate that agent-scope fences would issue for
// every chunk.
template <typename T>
__device__ __forceinline__ T coherent_load(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void coherent_store(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every vector memory operation of this wave has completed
// (s_waitcnt vmcnt(0); expcnt and lgkmcnt left unconstrained).
__device__ __forceinline__ void wait_vm_done() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
}

__device__ __forceinline__ void wait_at_least(const uint32_t *p, uint32_t need) {
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need)
        __builtin_amdgcn_s_sleep(2);
}

// slot index (10x10 grid, jl fastest) of the li-th non-corner staged line
__device__ __forceinline__ int staged_slot(int li) {
    if (li < 8) return li + 1;                       // kl = 0, jl = 1..8
    if (li < 88) return 10 + (li - 8);               // kl = 1..8, jl = 0..9
    return 90 + (li - 88) + 1;                       // kl = 9, jl = 1..8
}

// One work item: sweep tau of bundle (J, K) of one grid, marched along x.
template <typename T, bool HAS_A, bool HAS_F>
__device__ __forceinline__ void gs_item(const GsJob<T> &A, int tau, int J, int K, T *ring,
                                        T *fring) {
    const int lane = threadIdx.x;
    const int kk = lane & 7, jj = lane >> 3;  // kk fastest: conflict-free LDS
    const int d = jj + kk;                    // skew of this lane's line
    constexpr int GS_S = GsLds<T>::S;  // LDS stride per staged line
    const int own = (kk + 1) * 10 + (jj + 1) - GS_SLOT0;  // ring slot of this lane's line
    const int fown = jj * 8 + kk;
    const int h = A.h;
        const int j0 = h + 8 * J, k0 = h + 8 * K;
        const int j = j0 + jj, k = k0 + kk;
        const bool active = (j < h + A.ny) && (k < h + A.nz);
        const int nbun = A.nj * A.nk;
        const int me = K * A.nj + J;
        uint32_t *Pcur = A.progress + (size_t)tau * nbun;          // this sweep
        uint32_t *Pprev = Pcur - nbun;                              // previous sweep

        // Per-item staging tables: lane-constant line pointers and LDS offsets
        // of the 12 (load) and 8 (store) elements this lane moves per chunk.
        // Element m of a chunk is position 8c + xoff - lsh[m] of its line, where
        // lsh is that line's shift (the same for every item touching the line,
        // so producers and consumers agree on what "chunk c" holds).
        const T *lsrc[12];
        int lring[12];
        bool lok[12];
        int lsh[12];
#pragma unroll
        for (int m = 0; m < 12; ++m) {
            const int e = lane + 64 * m;
            const int slot = staged_slot(e >> 3);
            const int jl = slot % 10, kl = slot / 10;
            const int jg = j0 - 1 + jl, kg = k0 - 1 + kl;
            lok[m] = jg <= h + A.ny && kg <= h + A.nz;
            const T *l0 = A.u + (int64_t)kg * A.plane + (int64_t)jg * A.px + h;
            lsh[m] = (int)((reinterpret_cast<uintptr_t>(l0) / sizeof(T)) & (GS_C - 1));
            lsrc[m] = l0 + (e & 7) - lsh[m];
            lring[m] = (slot - GS_SLOT0) * GS_S;
        }
        T *sdst[8];
        int sring[8];
        bool sok[8];
        int ssh[8];
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            const int e = lane + 64 * m;
            const int li = e >> 3;
            const int jq = li & 7, kq = li >> 3;
            const int jg = j0 + jq, kg = k0 + kq;
            sok[m] = jg < h + A.ny && kg < h + A.nz;
            T *l0 = A.u + (int64_t)kg * A.plane + (int64_t)jg * A.px + h;
            ssh[m] = (int)((reinterpret_cast<uintptr_t>(l0) / sizeof(T)) & (GS_C - 1));
            sdst[m] = l0 + (e & 7) - ssh[m];
            sring[m] = ((kq + 1) * 10 + (jq + 1) - GS_SLOT0) * GS_S;
        }
        // f (interior-only, its own row pitch) is staged with its own line
        // alignment: f chunk c covers [8c - fsh, 8c + 8 - fsh) of the line.
        int fsh[HAS_F ? 8 : 1];
        if constexpr (HAS_F) {
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const int li = (lane + 64 * m) >> 3;
                const int jg = j0 + (li & 7), kg = k0 + (li >> 3);
                const T *f0 = A.f + ((int64_t)(kg - h) * A.ny + (jg - h)) * A.nx;
                fsh[m] = (int)((reinterpret_cast<uintptr_t>(f0) / sizeof(T)) & (GS_C - 1));
            }
        }
        const int xoff = lane & 7;  // chunk-relative position of every element

        // Dependencies: own bundle at tau-1, (J+1,K) and (J,K+1) at tau-1 (old
        // values), (J-1,K) and (J,K-1) at tau (fresh values).  The five polls
        // of one chunk are issued together and only the unsatisfied ones spin.
        // (Carrying the last seen values from chunk to chunk keeps five more
        // registers live through the sweep and measured markedly slower.)
        const uint32_t *dep[5] = {Pprev + me, Pprev + me + 1, Pprev + me + A.nj, Pcur + me - 1,
                                  Pcur + me - A.nj};
        const bool has[5] = {tau > 0, tau > 0 && J + 1 < A.nj, tau > 0 && K + 1 < A.nk, J > 0,
                             K > 0};
        auto wait_chunk = [&](int c) {
            if (c >= A.ncs) return;  // only positions >= nx: never written
            const uint32_t need = (uint32_t)c + 1u;
            uint32_t v[5];
#pragma unroll
            for (int q = 0; q < 5; ++q)
                v[q] = has[q] ? __hip_atomic_load(dep[q], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)
                              : need;
#pragma unroll
            for (int q = 0; q < 5; ++q)
                while (v[q] < need) {
                    __builtin_amdgcn_s_sleep(2);
                    v[q] = __hip_atomic_load(dep[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            // keep the coherent data loads below after the counter checks
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        };
        // Chunk staging is software-pipelined: the global loads of chunk c are
        // issued one block before c is written to LDS, and the stores of a
        // finished chunk are published one block after they were issued, so
        // neither latency stalls the sweep.
        T pf[12];  // chunk in flight from global memory
        T fpf[HAS_F ? 8 : 1];
        auto issue_load = [&](int c) {
            const int q = c * GS_C + xoff;
#pragma unroll
            for (int m = 0; m < 12; ++m) {
                const int i = q - lsh[m];  // 0..nx: interior and the x+ ghost
                pf[m] = (lok[m] && (unsigned)i <= (unsigned)A.nx)
                            ? coherent_load(lsrc[m] + c * GS_C)
                            : T(0);
            }
            if constexpr (HAS_F) {
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int e = lane + 64 * m;
                    const int li = e >> 3;
                    const int jq = li & 7, kq = li >> 3;
                    const int jg = j0 + jq, kg = k0 + kq;
                    const int i = q - fsh[m];
                    fpf[m] = ((unsigned)i < (unsigned)A.nx && sok[m])
                                 ? A.f[((int64_t)(kg - h) * A.ny + (jg - h)) * A.nx + i]
                                 : T(0);
                }
            }
        };
        auto commit_load = [&](int c) {  // prefetched chunk -> LDS ring
            const int q = c * GS_C + xoff;
#pragma unroll
            for (int m = 0; m < 12; ++m) ring[lring[m] + ((q - lsh[m]) & (GS_RING - 1))] = pf[m];
            if constexpr (HAS_F) {
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int li = (lane + 64 * m) >> 3;
                    fring[((li & 7) * 8 + (li >> 3)) * GS_S + ((q - fsh[m]) & (GS_RING - 1))] =
                        fpf[m];
                }
            }
        };
        auto issue_store = [&](int c) {  // LDS ring -> global (not yet published)
            const int q = c * GS_C + xoff;
            T v[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) v[m] = ring[sring[m] + ((q - ssh[m]) & (GS_RING - 1))];
#pragma unroll
            for (int m = 0; m < 8; ++m)
                if (sok[m] && (unsigned)(q - ssh[m]) < (unsigned)A.nx)
                    coherent_store(sdst[m] + c * GS_C, v[m]);
        };
        auto publish = [&](int c) {  // stores of chunk c have completed
            if (lane == 0)
                __hip_atomic_store(Pcur + me, (uint32_t)c + 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        };

        // x- ghost of this lane's line
        T xm = T(0);
        if (active) xm = A.u[(int64_t)k * A.plane + (int64_t)j * A.px + (h - 1)];

        // prologue: chunks 0 and 1 in LDS, chunk 2 in flight
        wait_chunk(0);
        issue_load(0);
        commit_load(0);
        if (A.ncl > 1) {
            wait_chunk(1);
            issue_load(1);
            commit_load(1);
        }
        if (A.ncl > 2) {
            wait_chunk(2);
            issue_load(2);
        }
        for (int b = 0; b < A.nb; ++b) {
#pragma unroll
            for (int st = 0; st < GS_C; ++st) {
                const int i = b * GS_C + st - d;
                if (active && i >= 0 && i < A.nx) {
                    const int p = i & (GS_RING - 1);
                    const T xp = ring[own * GS_S + ((i + 1) & (GS_RING - 1))];
                    const T ym = ring[(own - 1) * GS_S + p];
                    const T yp = ring[(own + 1) * GS_S + p];
                    const T zm = ring[(own - 10) * GS_S + p];
                    const T zp = ring[(own + 10) * GS_S + p];
                    T s = xm + xp;
                    s = s + ym;
                    s = s + yp;
                    s = s + zm;
                    s = s + zp;
                    T v;
                    if constexpr (HAS_A)
                        v = (A.a * ring[own * GS_S + p]) + (A.b * s);
                    else
                        v = A.b * s;
                    if constexpr (HAS_F) v = v + (A.g * fring[fown * GS_S + p]);
                    ring[own * GS_S + p] = v;
                    xm = v;
                }
                // LDS traffic of one wave is processed in order; keep the
                // compiler from moving this step's write after the next reads
                __builtin_amdgcn_wave_barrier();
            }
            // block boundary.  Chunk b-2 is final (the trailing lane, skew 14,
            // is past it); chunk b+2 must be in LDS before block b+1.
            wait_vm_done();                       // stores of b-3, loads of b+2
            if (b - 3 >= 0 && b - 3 < A.ncs) publish(b - 3);
            if (b - 2 >= 0 && b - 2 < A.ncs) issue_store(b - 2);  // reads slot of b+2 first
            if (b + 2 < A.ncl) commit_load(b + 2);
            if (b + 3 < A.ncl) {
                wait_chunk(b + 3);
                issue_load(b + 3);
            }
        }
        // drain: publish the last issued stores, then store the rest
        wait_vm_done();
        if (A.nb - 3 >= 0 && A.nb - 3 < A.ncs) publish(A.nb - 3);
        for (int cs = max(0, A.nb - 2); cs < A.ncs; ++cs) {
            issue_store(cs);
            wait_vm_done();
            publish(cs);
        }
}

template <typename T, bool HAS_A, bool HAS_F>
__global__ void __launch_bounds__(64) gs_wavefront_kernel(GsArgs<T> G) {
    __shared__ T ring[GsLds<T>::RING_LEN];
    __shared__ T fring[HAS_F ? GsLds<T>::FRING_LEN : 1];
    for (;;) {
        uint32_t t = 0;
        if (threadIdx.x == 0)
            t = __hip_atomic_fetch_add(G.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = __shfl(t, 0, 64);
        if (t >= G.nitems) break;
        const uint32_t it = G.items[t];
        gs_item<T, HAS_A, HAS_F>(G.job, (int)(it >> 20), (int)((it >> 10) & 1023u),
                                 (int)(it & 1023u), ring, fring);
    }
}

template <typename T, bool HAS_A, bool HAS_F>
__global__ void __launch_bounds__(64) gs_batch_kernel(GsBatchArgs<T> G) {
    __shared__ T ring[GsLds<T>::RING_LEN];
    __shared__ T fring[HAS_F ? GsLds<T>::FRING_LEN : 1];
    for (;;) {
        uint32_t t = 0;
        if (threadIdx.x == 0)
            t = __hip_atomic_fetch_add(G.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        t = __shfl(t, 0, 64);
        if (t >= G.nitems) break;
        const uint64_t it = G.items[t];
        const GsJob<T> job = G.jobs[(int)(it >> 48)];
        gs_item<T, HAS_A, HAS_F>(job, (int)((it >> 32) & 0xffffu), (int)((it >> 16) & 0xffffu),
                                 (int)(it & 0xffffu), ring, fring);
    }
}

__global__ void gs_reset_kernel(uint32_t *progress, int n, uint32_t *ticket) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        progress[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0u;
}

// ---- host side: item tables and flag buffers (library-owned) ----

struct GsBuffers {
    uint32_t *progress = nullptr;
    uint32_t *ticket = nullptr;
    int cap = 0;
};

std::mutex g_gs_mu;
// Progress counters and the ticket are reset at the start of every launch, so
// launches that may run concurrently (different streams) get separate ones;
// launches on one stream are ordered and can share them.
std::map<std::pair<int, hipStream_t>, GsBuffers> g_gs_bufs;
std::map<std::tuple<int, int, int, int>, uint32_t *> g_gs_items;  // (dev, nj, nk, S)

hipError_t get_items(int dev, int nj, int nk, int S, uint32_t **out, uint32_t *count) {
    auto key = std::make_tuple(dev, nj, nk, S);
    *count = (uint32_t)S * nj * nk;
    auto itx = g_gs_items.find(key);
    if (itx != g_gs_items.end()) {
        *out = itx->second;
        return hipSuccess;
    }
    std::vector<uint32_t> items;
    items.reserve(*count);
    const int kmax = 2 * (S - 1) + (nj - 1) + (nk - 1);
    for (int key2 = 0; key2 <= kmax; ++key2)
        for (int tau = 0; tau < S; ++tau) {
            const int rest = key2 - 2 * tau;
            if (rest < 0) break;
            for (int J = 0; J < nj; ++J) {
                const int K = rest - J;
                if (K < 0) break;
                if (K >= nk) continue;
                items.push_back(((uint32_t)tau << 20) | ((uint32_t)J << 10) | (uint32_t)K);
            }
        }
    uint32_t *d = nullptr;
    hipError_t e = hipMalloc(&d, items.size() * sizeof(uint32_t));
    if (e != hipSuccess) return e;
    e = hipMemcpy(d, items.data(), items.size() * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return e;
    }
    g_gs_items[key] = d;
    *out = d;
    return hipSuccess;
}

hipError_t get_bufs(int dev, hipStream_t s, int ncounters, GsBuffers **out) {
    GsBuffers &B = g_gs_bufs[std::make_pair(dev, s)];
    if (B.cap < ncounters) {
        if (B.progress) (void)hipFree(B.progress);
        if (B.ticket) (void)hipFree(B.ticket);
        B.progress = nullptr;
        B.ticket = nullptr;
        B.cap = 0;
        hipError_t e = hipMalloc(&B.progress, (size_t)ncounters * sizeof(uint32_t));
        if (e != hipSuccess) return e;
        e = hipMalloc(&B.ticket, 256);
        if (e != hipSuccess) return e;
        B.cap = ncounters;
    }
    *out = &B;
    return hipSuccess;
}

template <typename T>
GsJob<T> make_job(const Geom &g, void *u, const void *f, double a, double b, double gw,
                  uint32_t *progress) {
    GsJob<T> A;
    A.u = static_cast<T *>(u);
    A.f = static_cast<const T *>(f);
    A.px = g.px;
    A.plane = g.plane();
    A.nx = g.nx; A.ny = g.ny; A.nz = g.nz; A.h = g.h;
    A.a = (T)a; A.b = (T)b; A.g = (T)gw;
    A.nj = (g.ny + 7) / 8;
    A.nk = (g.nz + 7) / 8;
    // with line shifts 0..7: stores reach position nx-1, loads the x+ ghost nx
    A.ncs = (g.nx + GS_C - 2) / GS_C + 1;
    A.ncl = (g.nx + GS_C - 1) / GS_C + 1;
    A.nb = (g.nx + 14 + GS_C - 1) / GS_C;
    A.progress = progress;
    return A;
}

int device_cus(int dev) {
    // cached on first use; concurrent first calls store the same value
    static std::atomic<int> cached[64];
    if (dev < 0 || dev >= 64) return 256;
    int ncu = cached[dev].load(std::memory_order_relaxed);
    if (ncu == 0) {
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                hipSuccess || ncu < 1)
            ncu = 256;
        cached[dev].store(ncu, std::memory_order_relaxed);
    }
    return ncu;
}

template <typename K>
int per_cu_occupancy(K kfn) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kfn),
                                                     64, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    return per_cu;
}

template <typename T, bool HAS_A, bool HAS_F>
hipError_t launch_gs_t(const Geom &g, void *u, const void *f, double a, double b, double gw,
                       int S, hipStream_t s, std::string *err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    GsArgs<T> G;
    G.job = make_job<T>(g, u, f, a, b, gw, nullptr);
    const int nj = G.job.nj, nk = G.job.nk;
    if (nj > 1024 || nk > 1024 || S > 4095) {
        if (err) *err = "Gauss-Seidel grid too large for one launch (ny, nz <= 8192)";
        return hipErrorInvalidValue;
    }
    {
        std::lock_guard<std::mutex> lk(g_gs_mu);
        GsBuffers *B = nullptr;
        e = get_bufs(dev, s, S * nj * nk, &B);
        if (e != hipSuccess) return e;
        uint32_t *items = nullptr;
        e = get_items(dev, nj, nk, S, &items, &G.nitems);
        if (e != hipSuccess) return e;
        G.items = items;
        G.job.progress = B->progress;
        G.ticket = B->ticket;
    }
    hipLaunchKernelGGL(gs_reset_kernel, dim3(256), dim3(256), 0, s, G.job.progress, S * nj * nk,
                       G.ticket);
    static std::atomic<int> per_cu_cached{0};
    int per_cu = per_cu_cached.load(std::memory_order_relaxed);
    if (per_cu == 0) {
        per_cu = per_cu_occupancy(gs_wavefront_kernel<T, HAS_A, HAS_F>);
        per_cu_cached.store(per_cu, std::memory_order_relaxed);
    }
    int grid = per_cu * device_cus(dev);
    if ((uint32_t)grid > G.nitems) grid = (int)G.nitems;
    hipLaunchKernelGGL((gs_wavefront_kernel<T, HAS_A, HAS_F>), dim3(grid), dim3(64), 0, s, G);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gs_any(const Geom &g, void *u, const void *f, double a, double b, double gw,
                         int S, hipStream_t s, std::string *err) {
    const bool ha = a != 0.0, hf = f != nullptr;
    if (ha && hf) return launch_gs_t<T, true, true>(g, u, f, a, b, gw, S, s, err);
    if (ha) return launch_gs_t<T, true, false>(g, u, f, a, b, gw, S, s, err);
    if (hf) return launch_gs_t<T, false, true>(g, u, f, a, b, gw, S, s, err);
    return launch_gs_t<T, false, false>(g, u, f, a, b, gw, S, s, err);
}

// ---- batched launch (job service) ----

template <typename T, bool HAS_A, bool HAS_F>
hipError_t launch_gs_batch_t(const std::vector<GsBatchItem> &items, GsBatchWork &w,
                             hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const size_t nj_ = items.size();
    // progress counters: one block per job, [sweeps][bundles]
    size_t ncount = 0;
    std::vector<size_t> off(nj_);
    for (size_t j = 0; j < nj_; ++j) {
        const int nj = (items[j].g.ny + 7) / 8, nk = (items[j].g.nz + 7) / 8;
        off[j] = ncount;
        ncount += (size_t)items[j].sweeps * nj * nk;
    }
    // merged item list in key order 2*tau + J + K (ties: by job)
    w.items.clear();
    int kmax = 0;
    for (const auto &it : items) {
        const int nj = (it.g.ny + 7) / 8, nk = (it.g.nz + 7) / 8;
        kmax = std::max(kmax, 2 * (it.sweeps - 1) + nj - 1 + nk - 1);
    }
    for (int key = 0; key <= kmax; ++key)
        for (size_t j = 0; j < nj_; ++j) {
            const int nj = (items[j].g.ny + 7) / 8, nk = (items[j].g.nz + 7) / 8;
            for (int tau = 0; tau < items[j].sweeps; ++tau) {
                const int rest = key - 2 * tau;
                if (rest < 0) break;
                for (int J = 0; J < nj; ++J) {
                    const int K = rest - J;
                    if (K < 0) break;
                    if (K >= nk) continue;
                    w.items.push_back(((uint64_t)j << 48) | ((uint64_t)tau << 32) |
                                      ((uint64_t)J << 16) | (uint64_t)K);
                }
            }
        }
    const size_t jobs_bytes = nj_ * sizeof(GsJob<T>);
    const size_t items_bytes = w.items.size() * sizeof(uint64_t);
    // one device buffer: jobs | items | progress counters | ticket, each part
    // starting on a 256-byte boundary
    auto up256 = [](size_t n) { return (n + 255) / 256 * 256; };
    const size_t off_items = up256(jobs_bytes);
    const size_t off_prog = off_items + up256(items_bytes);
    const size_t off_ticket = off_prog + up256(ncount * sizeof(uint32_t));
    const size_t need = off_ticket + 256;
    if (w.dev_bytes < need) {
        if (w.dev) (void)hipFree(w.dev);
        w.dev = nullptr;
        w.dev_bytes = 0;
        e = hipMalloc(&w.dev, need * 2);
        if (e != hipSuccess) return e;
        w.dev_bytes = need * 2;
    }
    char *base = static_cast<char *>(w.dev);
    GsJob<T> *djobs = reinterpret_cast<GsJob<T> *>(base);
    uint64_t *ditems = reinterpret_cast<uint64_t *>(base + off_items);
    uint32_t *dprog = reinterpret_cast<uint32_t *>(base + off_prog);
    uint32_t *dticket = reinterpret_cast<uint32_t *>(base + off_ticket);
    w.jobs_host.resize(jobs_bytes);
    GsJob<T> *hj = reinterpret_cast<GsJob<T> *>(w.jobs_host.data());
    for (size_t j = 0; j < nj_; ++j)
        hj[j] = make_job<T>(items[j].g, items[j].u, items[j].f, items[j].a, items[j].b,
                            items[j].gw, dprog + off[j]);
    e = hipMemcpyAsync(djobs, hj, jobs_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(ditems, w.items.data(), items_bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gs_reset_kernel, dim3(256), dim3(256), 0, s, dprog, (int)ncount, dticket);
    GsBatchArgs<T> G;
    G.jobs = djobs;
    G.nitems = (uint32_t)w.items.size();
    G.items = ditems;
    G.ticket = dticket;
    static std::atomic<int> per_cu_cached{0};
    int per_cu = per_cu_cached.load(std::memory_order_relaxed);
    if (per_cu == 0) {
        per_cu = per_cu_occupancy(gs_batch_kernel<T, HAS_A, HAS_F>);
        per_cu_cached.store(per_cu, std::memory_order_relaxed);
    }
    int grid = per_cu * device_cus(dev);
    if ((uint32_t)grid > G.nitems) grid = (int)G.nitems;
    hipLaunchKernelGGL((gs_batch_kernel<T, HAS_A, HAS_F>), dim3(grid), dim3(64), 0, s, G);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gs_batch_any(bool ha, bool hf, const std::vector<GsBatchItem> &items,
                               GsBatchWork &w, hipStream_t s) {
    if (ha && hf) return launch_gs_batch_t<T, true, true>(items, w, s);
    if (ha) return launch_gs_batch_t<T, true, false>(items, w, s);
    if (hf) return launch_gs_batch_t<T, false, true>(items, w, s);
    return launch_gs_batch_t<T, false, false>(items, w, s);
}

}  // namespace

hipError_t launch_gs(bool fp32, const Geom &g, void *u, const void *f, double a, double b,
                     double gw, int sweeps, hipStream_t s, std::string *err) {
    return fp32 ? launch_gs_any<float>(g, u, f, a, b, gw, sweeps, s, err)
                : launch_gs_any<double>(g, u, f, a, b, gw, sweeps, s, err);
}

hipError_t launch_gs_batch(bool fp32, bool has_a, bool has_f,
                           const std::vector<GsBatchItem> &items, GsBatchWork &w, hipStream_t s) {
    if (items.empty()) return hipSuccess;
    return fp32 ? launch_gs_batch_any<float>(has_a, has_f, items, w, s)
                : launch_gs_batch_any<double>(has_a, has_f, items, w, s);
}

GsBatchWork::~GsBatchWork() {
    if (dev) (void)hipFree(dev);
}

}  // namespace stk
