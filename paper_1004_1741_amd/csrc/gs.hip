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

// Control block of one device.
// abort: set by a wave that gave up waiting, or by the host
// (stencil_gs_abort); every wait and every ticket fetch checks it, so all
// waves then finish their items without waiting and exit.  status: bit 0 is
// set by a wave that gave up; read and cleared by the host (stencil_sync).
struct GsCtl {
    uint32_t abort;
    uint32_t status;
    uint32_t pad_[62];
};

template <typename T>
struct GsArgs {
    GsJob<T> job;
    uint32_t nitems;
    const uint32_t *items;   // (tau << 20) | (J << 10) | K, topologically ordered
    uint32_t *ticket;
    GsCtl *ctl;
    uint32_t spin_limit;     // polls of one wait before giving up
};

// Batched launch: items of several jobs merged in key order; each item is
// (job << 48) | (tau << 32) | (J << 16) | K.
template <typename T>
struct GsBatchArgs {
    const GsJob<T> *jobs;
    uint32_t nitems;
    const uint64_t *items;
    uint32_t *ticket;
    GsCtl *ctl;
    uint32_t spin_limit;
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

// A wave that gives up raises the device's abort word (seen by every other
// wait within 64 polls) and records the failure for the host.
__device__ __forceinline__ void give_up(GsCtl *ctl) {
    if (threadIdx.x == 0) {
        __hip_atomic_store(&ctl->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_or(&ctl->status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __forceinline__ bool aborted(const GsCtl *ctl) {
    return __hip_atomic_load(&ctl->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u;
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
                                        T *fring, GsCtl *ctl, uint32_t spin_limit) {
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
        // Every wait is bounded: after spin_limit polls, or once the abort word
        // is raised, the wave gives up and runs the rest of the item without
        // waiting (its results are then invalid and the launch reports it).
        bool dead = false;
        auto wait_chunk = [&](int c) {
            if (c >= A.ncs || dead) return;  // c >= ncs: only positions >= nx, never written
            const uint32_t need = (uint32_t)c + 1u;
            uint32_t v[5];
#pragma unroll
            for (int q = 0; q < 5; ++q)
                v[q] = has[q] ? __hip_atomic_load(dep[q], __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT)
                              : need;
            uint32_t polls = 0;
#pragma unroll
            for (int q = 0; q < 5; ++q)
                while (v[q] < need) {
                    ++polls;
                    if (polls >= spin_limit || ((polls & 63u) == 0u && aborted(ctl))) {
                        give_up(ctl);
                        dead = true;
                        return;
                    }
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

// Next ticket for this wave, or nitems (stop) once the abort word is raised;
// a launch stopped that way reports it like a wait that gave up.
__device__ __forceinline__ uint32_t next_ticket(uint32_t *ticket, uint32_t nitems, GsCtl *ctl) {
    uint32_t t = 0;
    if (threadIdx.x == 0) {
        if (aborted(ctl)) {
            __hip_atomic_fetch_or(&ctl->status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            t = nitems;
        } else {
            t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    return __shfl(t, 0, 64);
}

template <typename T, bool HAS_A, bool HAS_F>
__global__ void __launch_bounds__(64) gs_wavefront_kernel(GsArgs<T> G) {
    __shared__ T ring[GsLds<T>::RING_LEN];
    __shared__ T fring[HAS_F ? GsLds<T>::FRING_LEN : 1];
    for (;;) {
        const uint32_t t = next_ticket(G.ticket, G.nitems, G.ctl);
        if (t >= G.nitems) break;
        const uint32_t it = G.items[t];
        gs_item<T, HAS_A, HAS_F>(G.job, (int)(it >> 20), (int)((it >> 10) & 1023u),
                                 (int)(it & 1023u), ring, fring, G.ctl, G.spin_limit);
    }
}

template <typename T, bool HAS_A, bool HAS_F>
__global__ void __launch_bounds__(64) gs_batch_kernel(GsBatchArgs<T> G) {
    __shared__ T ring[GsLds<T>::RING_LEN];
    __shared__ T fring[HAS_F ? GsLds<T>::FRING_LEN : 1];
    for (;;) {
        const uint32_t t = next_ticket(G.ticket, G.nitems, G.ctl);
        if (t >= G.nitems) break;
        const uint64_t it = G.items[t];
        const GsJob<T> job = G.jobs[(int)(it >> 48)];
        gs_item<T, HAS_A, HAS_F>(job, (int)((it >> 32) & 0xffffu), (int)((it >> 16) & 0xffffu),
                                 (int)(it & 0xffffu), ring, fring, G.ctl, G.spin_limit);
    }
}

__global__ void gs_reset_kernel(uint32_t *progress, int64_t n, uint32_t *ticket) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        progress[i] = 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) *ticket = 0u;
}

// ---- item table, built on the device for every launch ----
// Items (tau, J, K) are ordered by key = 2*tau + J + K, then tau, then J.
// Bundles J of a "rest" r = key - 2*tau run over [max(0, r - nk + 1),
// min(nj - 1, r)].
__device__ __forceinline__ int rest_lo(int r, int nk) { return r - (nk - 1) > 0 ? r - (nk - 1) : 0; }
__device__ __forceinline__ int rest_count(int r, int nj, int nk) {
    if (r < 0) return 0;
    const int hi = r < nj - 1 ? r : nj - 1;
    const int lo = rest_lo(r, nk);
    return hi >= lo ? hi - lo + 1 : 0;
}
// first tau whose rest r = key - 2 tau can be a valid J + K (r <= nj + nk - 2)
__device__ __forceinline__ int tau_first(int key, int nj, int nk) {
    const int d = key - (nj + nk - 2);
    return d > 0 ? (d + 1) / 2 : 0;
}

// One block: prefix[key] = number of items with a smaller key; clears the
// ticket.  nkeys = 2 (S - 1) + nj + nk - 1.
__global__ void __launch_bounds__(1024) gs_prefix_kernel(int S, int nj, int nk,
                                                         uint32_t *__restrict__ prefix,
                                                         uint32_t *__restrict__ ticket) {
    __shared__ uint32_t part[1024];
    const int nkeys = 2 * (S - 1) + nj + nk - 1;
    const int per = (nkeys + 1023) / 1024;
    const int k0 = threadIdx.x * per;
    uint32_t local = 0;
    for (int k = k0; k < k0 + per && k < nkeys; ++k) {
        const int t1 = min(S - 1, k / 2);
        for (int tau = tau_first(k, nj, nk); tau <= t1; ++tau)
            local += (uint32_t)rest_count(k - 2 * tau, nj, nk);
    }
    part[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {  // inclusive scan of the chunk sums
        const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0u;
    for (int k = k0; k < k0 + per && k < nkeys; ++k) {
        prefix[k] = run;
        const int t1 = min(S - 1, k / 2);
        for (int tau = tau_first(k, nj, nk); tau <= t1; ++tau)
            run += (uint32_t)rest_count(k - 2 * tau, nj, nk);
    }
    if (threadIdx.x == 0) {
        prefix[nkeys] = part[1023];
        *ticket = 0u;
    }
}

// One thread per item: writes it at its position in key order and clears its
// progress counter.
__global__ void __launch_bounds__(256) gs_items_kernel(int S, int nj, int nk,
                                                       const uint32_t *__restrict__ prefix,
                                                       uint32_t *__restrict__ items,
                                                       uint32_t *__restrict__ progress) {
    const int64_t n = (int64_t)S * nj * nk;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int nb = nj * nk;
    const int tau = (int)(i / nb);
    const int rem = (int)(i - (int64_t)tau * nb);
    const int K = rem / nj, J = rem - K * nj;
    const int key = 2 * tau + J + K;
    uint32_t pos = prefix[key];
    for (int t = tau_first(key, nj, nk); t < tau; ++t) pos += (uint32_t)rest_count(key - 2 * t, nj, nk);
    pos += (uint32_t)(J - rest_lo(key - 2 * tau, nk));
    items[pos] = ((uint32_t)tau << 20) | ((uint32_t)J << 10) | (uint32_t)K;
    progress[i] = 0u;
}

// ---- per-device control block ----
// One GsCtl per device, a static device variable.  Host code never uses the
// variable's name as an address: the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
__device__ GsCtl gs_ctl;

__global__ void gs_ctl_clear_kernel(GsCtl *ctl) {
    if (threadIdx.x == 0) {
        ctl->abort = 0u;
        ctl->status = 0u;
    }
}

std::mutex g_ctl_mu;
GsCtl *g_ctl_ptr[64];                       // device address of gs_ctl, per device
hipStream_t g_ctl_stream[64];               // for host writes while kernels run
std::atomic<uint32_t> g_spin_limit{1u << 24};

// Device address of this device's control block (looked up and cleared on
// first use; the clear is a kernel on stream s, ordered before the caller's
// work).
hipError_t device_ctl(int dev, hipStream_t s, GsCtl **out) {
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_ctl_mu);
    if (!g_ctl_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(gs_ctl));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(gs_ctl_clear_kernel, dim3(1), dim3(64), 0, s, static_cast<GsCtl *>(p));
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        g_ctl_ptr[dev] = static_cast<GsCtl *>(p);
    }
    *out = g_ctl_ptr[dev];
    return hipSuccess;
}

// Workspace of one launch of S sweeps over nj x nk bundles, laid out from
// `base` (may be nullptr to only compute the size).
struct GsWork {
    uint32_t *progress, *ticket, *prefix, *items;
    size_t bytes;
};
GsWork gs_work_layout(int S, int nj, int nk, unsigned char *base) {
    auto up = [](size_t n) { return (n + 255) / 256 * 256; };
    const size_t nitems = (size_t)S * nj * nk;
    const size_t nkeys = (size_t)2 * (S - 1) + nj + nk - 1;
    const size_t o_ticket = up(nitems * 4);
    const size_t o_prefix = o_ticket + 256;
    const size_t o_items = o_prefix + up((nkeys + 1) * 4);
    GsWork w;
    w.bytes = o_items + up(nitems * 4);
    w.progress = reinterpret_cast<uint32_t *>(base);
    w.ticket = reinterpret_cast<uint32_t *>(base + o_ticket);
    w.prefix = reinterpret_cast<uint32_t *>(base + o_prefix);
    w.items = reinterpret_cast<uint32_t *>(base + o_items);
    return w;
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

// One launch of S sweeps.  ws: workspace of gs_work_layout(S, nj, nk) bytes
// on the device; the item table is built there by two small kernels.
template <typename T, bool HAS_A, bool HAS_F>
hipError_t launch_gs_t(const Geom &g, void *u, const void *f, double a, double b, double gw,
                       int S, GsCtl *ctl, unsigned char *ws, hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    GsArgs<T> G;
    G.job = make_job<T>(g, u, f, a, b, gw, nullptr);
    const int nj = G.job.nj, nk = G.job.nk;
    const GsWork w = gs_work_layout(S, nj, nk, ws);
    const int64_t nitems = (int64_t)S * nj * nk;
    hipLaunchKernelGGL(gs_prefix_kernel, dim3(1), dim3(1024), 0, s, S, nj, nk, w.prefix, w.ticket);
    hipLaunchKernelGGL(gs_items_kernel, dim3((unsigned)((nitems + 255) / 256)), dim3(256), 0, s, S,
                       nj, nk, (const uint32_t *)w.prefix, w.items, w.progress);
    G.nitems = (uint32_t)nitems;
    G.items = w.items;
    G.ticket = w.ticket;
    G.job.progress = w.progress;
    G.ctl = ctl;
    G.spin_limit = g_spin_limit.load(std::memory_order_relaxed);
    static std::atomic<int> per_cu_cached{0};
    int per_cu = per_cu_cached.load(std::memory_order_relaxed);
    if (per_cu == 0) {
        per_cu = per_cu_occupancy(gs_wavefront_kernel<T, HAS_A, HAS_F>);
        per_cu_cached.store(per_cu, std::memory_order_relaxed);
    }
    int64_t grid = (int64_t)per_cu * device_cus(dev);
    if (grid > nitems) grid = nitems;
    hipLaunchKernelGGL((gs_wavefront_kernel<T, HAS_A, HAS_F>), dim3((unsigned)grid), dim3(64), 0,
                       s, G);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gs_any(const Geom &g, void *u, const void *f, double a, double b, double gw,
                         int S, GsCtl *ctl, unsigned char *ws, hipStream_t s) {
    const bool ha = a != 0.0, hf = f != nullptr;
    if (ha && hf) return launch_gs_t<T, true, true>(g, u, f, a, b, gw, S, ctl, ws, s);
    if (ha) return launch_gs_t<T, true, false>(g, u, f, a, b, gw, S, ctl, ws, s);
    if (hf) return launch_gs_t<T, false, true>(g, u, f, a, b, gw, S, ctl, ws, s);
    return launch_gs_t<T, false, false>(g, u, f, a, b, gw, S, ctl, ws, s);
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
    if (ncount > 0xffffffffull || w.items.size() > 0xffffffffull) return hipErrorInvalidValue;
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
    hipLaunchKernelGGL(gs_reset_kernel, dim3(256), dim3(256), 0, s, dprog, (int64_t)ncount,
                       dticket);
    GsBatchArgs<T> G;
    G.jobs = djobs;
    G.nitems = (uint32_t)w.items.size();
    G.items = ditems;
    G.ticket = dticket;
    e = device_ctl(dev, s, &G.ctl);
    if (e != hipSuccess) return e;
    G.spin_limit = g_spin_limit.load(std::memory_order_relaxed);
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
                     double gw, int sweeps, hipStream_t s) {
    if (sweeps < 1 || sweeps > 4095) return hipErrorInvalidValue;
    if ((int64_t)sweeps * ((g.ny + 7) / 8) * ((g.nz + 7) / 8) >= ((int64_t)1 << 31))
        return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    GsCtl *ctl = nullptr;
    e = device_ctl(dev, s, &ctl);
    if (e != hipSuccess) return e;
    const int nj = (g.ny + 7) / 8, nk = (g.nz + 7) / 8;
    // stream-ordered workspace, returned to the stream's pool after the launch
    const size_t bytes = gs_work_layout(sweeps, nj, nk, nullptr).bytes;
    void *ws = nullptr;
    e = hipMallocAsync(&ws, bytes, s);
    if (e != hipSuccess) return e;
    e = fp32 ? launch_gs_any<float>(g, u, f, a, b, gw, sweeps, ctl,
                                    static_cast<unsigned char *>(ws), s)
             : launch_gs_any<double>(g, u, f, a, b, gw, sweeps, ctl,
                                     static_cast<unsigned char *>(ws), s);
    const hipError_t ef = hipFreeAsync(ws, s);
    return e != hipSuccess ? e : ef;
}

// ---- allocation-free variant: workspace in a static device array ----
// One array per device, held until the process ends.  Host code never uses
// the array's name as an address: the device address comes from
// hipGetSymbolAddress, looked up once per device with that device current.
// Every launch rebuilds its item table and clears its counters and ticket in
// this array (gs_prefix_kernel, gs_items_kernel), so nothing carries over
// from the previous call; calls that overlap on one device race for it.
static __device__ __align__(256) unsigned char scratch[GS_NOALLOC_BYTES];

static unsigned char *g_scratch_ptr[64];  // device address of scratch, per device

static hipError_t device_scratch(int dev, unsigned char **out) {
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_ctl_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t gs_workspace_bytes(int sweeps, int ny, int nz) {
    return gs_work_layout(sweeps, (ny + 7) / 8, (nz + 7) / 8, nullptr).bytes;
}

hipError_t launch_gs_noalloc(bool fp32, const Geom &g, void *u, const void *f, double a,
                             double b, double gw, int sweeps, hipStream_t s) {
    if (sweeps < 1 || sweeps > 4095) return hipErrorInvalidValue;
    if (gs_workspace_bytes(sweeps, g.ny, g.nz) > GS_NOALLOC_BYTES) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    GsCtl *ctl = nullptr;
    e = device_ctl(dev, s, &ctl);
    if (e != hipSuccess) return e;
    unsigned char *ws = nullptr;
    e = device_scratch(dev, &ws);
    if (e != hipSuccess) return e;
    return fp32 ? launch_gs_any<float>(g, u, f, a, b, gw, sweeps, ctl, ws, s)
                : launch_gs_any<double>(g, u, f, a, b, gw, sweeps, ctl, ws, s);
}

hipError_t gs_status(int dev, hipStream_t s, bool clear, uint32_t *status) {
    GsCtl *ctl = nullptr;
    hipError_t e = device_ctl(dev, s, &ctl);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    uint32_t st = 0;
    e = hipMemcpyAsync(&st, &ctl->status, sizeof(st), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (clear) {
        hipLaunchKernelGGL(gs_ctl_clear_kernel, dim3(1), dim3(64), 0, s, ctl);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
    }
    *status = st;
    return hipSuccess;
}

hipError_t gs_abort(int dev) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (dev != cur) {
        e = hipSetDevice(dev);
        if (e != hipSuccess) return e;
    }
    hipStream_t st = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_ctl_mu);
        if (!g_ctl_stream[dev]) e = hipStreamCreateWithFlags(&g_ctl_stream[dev], hipStreamNonBlocking);
        st = g_ctl_stream[dev];
    }
    GsCtl *ctl = nullptr;
    if (e == hipSuccess) e = device_ctl(dev, st, &ctl);
    // written on a stream of its own so that it lands while wavefront
    // launches on other streams are running
    static const uint32_t one = 1u;
    if (e == hipSuccess) e = hipMemcpyAsync(&ctl->abort, &one, sizeof(one), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (dev != cur) (void)hipSetDevice(cur);
    return e;
}

void gs_set_spin_limit(uint32_t polls) {
    g_spin_limit.store(polls ? polls : (1u << 24), std::memory_order_relaxed);
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
