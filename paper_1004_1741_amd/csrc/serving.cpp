// serving.cpp -- continuous-batching job service (smooth_* in stencil.h).
//
// Jobs are independent smoothing problems of uneven sizes.  Threads:
//   * scheduler: admits queued jobs while their device footprint fits the
//     pool (one hipMalloc of hbm_budget_bytes, first-fit sub-allocation) and
//     fewer than max_inflight are resident, then runs *iterations*: every
//     resident job whose input is on the device does its sweeps (all of them,
//     or at most sweeps_per_iteration) in rounds of batched launches, where
//     all jobs of the same kind share one launch (one Jacobi pass kernel per
//     dtype/t group and round, one merged-ticket Gauss-Seidel wavefront per
//     group).  Jobs admitted while an iteration runs join the next one, so
//     their work overlaps with the others' on the device (iteration-level
//     continuous batching);
//   * uploaders / downloaders (kIoThreads of each): host<->device copies of
//     job grids on their own streams, so copies overlap with the iterations
//     and with each other (a single copy thread is limited by the runtime's
//     staging of pageable host memory).
// Batched kernels run each job's tiles/items exactly as the single-grid
// kernels do, so a job's result does not depend on its batch companions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/stencil.h"
#include "internal.h"
#include "pool.h"

namespace stk {
namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

enum Phase { PH_QUEUED, PH_UPLOADING, PH_READY, PH_PASSES, PH_FINISH, PH_DOWNLOADING, PH_END };

struct Job {
    uint64_t id = 0;
    smooth_job spec{};
    int32_t state = SMOOTH_QUEUED;
    smooth_stats st{};
    Geom g{};
    bool gs = false, refined = false;
    uint64_t bytes = 0, off = 0;
    bool allocated = false;
    int bypassed = 0;
    double *u = nullptr, *s64 = nullptr;                   // FP64 grid (+ Jacobi scratch)
    float *r32 = nullptr, *e32 = nullptr, *s32 = nullptr;  // refined: defect, correction
    std::vector<int> plan;  // Jacobi passes
    size_t pass = 0;
    int parity = 0;         // Jacobi: 1 = current data in the second buffer
    int sweeps_done = 0;
    Phase ph = PH_QUEUED;
    const double *result = nullptr;  // device grid to download
    hipEvent_t ev_done = nullptr;    // compute finished
};

uint64_t footprint(const smooth_job &j) {
    const uint64_t N = (uint64_t)(j.nx + 2) * (j.ny + 2) * (j.nz + 2);
    const uint64_t n = (uint64_t)j.nx * j.ny * j.nz;
    uint64_t b = PoolAllocator::round_up(8 * N);  // u
    if (j.precision == SMOOTH_FP64) {
        if (j.method == SMOOTH_JACOBI) b += PoolAllocator::round_up(8 * N);  // scratch
    } else {
        b += PoolAllocator::round_up(4 * n) + PoolAllocator::round_up(4 * N);  // r32, e32
        if (j.method == SMOOTH_JACOBI) b += PoolAllocator::round_up(4 * N);    // s32
    }
    return b;
}

}  // namespace
}  // namespace stk

using namespace stk;

// host<->device copy threads per direction
constexpr int kIoThreads = 4;

struct smooth_ctx {
    smooth_config cfg{};
    void *pool = nullptr;
    PoolAllocator alloc;
    hipStream_t s_comp = nullptr;
    std::vector<hipStream_t> s_up, s_down;  // one per copy thread
    hipEvent_t ev_iter = nullptr;
    std::mutex mu;
    std::condition_variable cv;       // scheduler wake-ups
    std::condition_variable cv_io;    // uploader / downloader wake-ups
    std::condition_variable cv_done;  // a job reached a terminal state
    std::deque<Job *> pending;        // submitted, not admitted
    std::deque<Job *> to_upload;
    std::deque<Job *> to_download;
    std::vector<Job *> resident;      // admitted, not terminal
    std::map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_id = 1;
    bool stop = false, sched_done = false;
    std::thread th_sched;
    std::vector<std::thread> th_up, th_down;
    int64_t batches = 0, n_done = 0, n_failed = 0, n_canceled = 0;
    int max_resident = 0;
    std::map<int, std::pair<void *, size_t>> jac_tables;   // group -> device table
    std::map<int, std::unique_ptr<GsBatchWork>> gs_works;  // group -> workspace
};

namespace {

// terminal transition (mu held)
void finish(smooth_ctx *c, Job *j, int32_t state) {
    j->state = state;
    j->ph = PH_END;
    j->st.t_done_ns = now_ns();
    if (j->allocated) c->alloc.release(j->off, j->bytes);
    j->allocated = false;
    if (j->ev_done) {
        (void)hipEventDestroy(j->ev_done);
        j->ev_done = nullptr;
    }
    c->resident.erase(std::remove(c->resident.begin(), c->resident.end(), j),
                      c->resident.end());
    if (state == SMOOTH_DONE) ++c->n_done;
    if (state == SMOOTH_FAILED) ++c->n_failed;
    if (state == SMOOTH_CANCELED) ++c->n_canceled;
    c->cv_done.notify_all();
    c->cv.notify_all();
}

// Admission (mu held): FIFO, but a job that does not fit lets later ones
// pass at most 8 times (counted when a later job is actually admitted ahead
// of it); after that admission waits for it.
void admit(smooth_ctx *c) {
    std::vector<Job *> skipped;  // jobs ahead of the current one that did not fit
    for (auto it = c->pending.begin(); it != c->pending.end();) {
        if ((int)c->resident.size() >= c->cfg.max_inflight) break;
        Job *j = *it;
        uint64_t off = 0;
        if (!c->alloc.alloc(j->bytes, &off)) {
            if (j->bypassed >= 8) break;
            skipped.push_back(j);
            ++it;
            continue;
        }
        for (Job *sk : skipped) ++sk->bypassed;
        j->off = off;
        j->allocated = true;
        char *base = static_cast<char *>(c->pool) + off;
        const uint64_t N = (uint64_t)j->g.count(), n = (uint64_t)j->g.interior();
        uint64_t o = 0;
        j->u = reinterpret_cast<double *>(base + o);
        o += PoolAllocator::round_up(8 * N);
        if (!j->refined) {
            if (!j->gs) j->s64 = reinterpret_cast<double *>(base + o);
        } else {
            j->r32 = reinterpret_cast<float *>(base + o);
            o += PoolAllocator::round_up(4 * n);
            j->e32 = reinterpret_cast<float *>(base + o);
            o += PoolAllocator::round_up(4 * N);
            if (!j->gs) j->s32 = reinterpret_cast<float *>(base + o);
        }
        j->state = SMOOTH_RUNNING;
        j->st.t_admit_ns = now_ns();
        j->st.footprint_bytes = j->bytes;
        j->ph = PH_UPLOADING;
        c->resident.push_back(j);
        c->max_resident = std::max(c->max_resident, (int)c->resident.size());
        c->to_upload.push_back(j);
        c->cv_io.notify_all();
        it = c->pending.erase(it);
    }
}

void uploader(smooth_ctx *c, int k) {
    (void)hipSetDevice(c->cfg.device);
    std::unique_lock<std::mutex> lk(c->mu);
    for (;;) {
        c->cv_io.wait(lk, [&] { return c->sched_done || !c->to_upload.empty(); });
        if (c->to_upload.empty()) return;  // scheduler finished and nothing left
        Job *j = c->to_upload.front();
        c->to_upload.pop_front();
        const size_t bytes = (size_t)j->g.count() * sizeof(double);
        lk.unlock();
        hipError_t e =
            hipMemcpyAsync(j->u, j->spec.input_host, bytes, hipMemcpyHostToDevice, c->s_up[k]);
        if (e == hipSuccess) e = hipStreamSynchronize(c->s_up[k]);
        lk.lock();
        if (e != hipSuccess) {
            set_error(std::string("job upload: ") + hipGetErrorString(e));
            finish(c, j, SMOOTH_FAILED);
            continue;
        }
        j->ph = PH_READY;
        j->st.t_uploaded_ns = now_ns();
        c->cv.notify_all();
    }
}

void downloader(smooth_ctx *c, int k) {
    (void)hipSetDevice(c->cfg.device);
    std::unique_lock<std::mutex> lk(c->mu);
    for (;;) {
        c->cv_io.wait(lk, [&] { return c->sched_done || !c->to_download.empty(); });
        if (c->to_download.empty()) return;
        Job *j = c->to_download.front();
        c->to_download.pop_front();
        const size_t bytes = (size_t)j->g.count() * sizeof(double);
        lk.unlock();
        hipError_t e = hipEventSynchronize(j->ev_done);
        if (e == hipSuccess)
            e = hipMemcpyAsync(j->spec.output_host, j->result, bytes, hipMemcpyDeviceToHost,
                               c->s_down[k]);
        if (e == hipSuccess) e = hipStreamSynchronize(c->s_down[k]);
        lk.lock();
        if (e != hipSuccess) set_error(std::string("job download: ") + hipGetErrorString(e));
        finish(c, j, e == hipSuccess ? SMOOTH_DONE : SMOOTH_FAILED);
    }
}

struct JacGroup {
    bool fp32;
    int tb;
    bool ha, hf;
    std::vector<JacBatchItem> items;
    std::vector<Job *> jobs;
    std::vector<unsigned char> staging;
};
struct GsGroup {
    bool fp32, ha, hf;
    std::vector<GsBatchItem> items;
    std::vector<Job *> jobs;
    std::vector<int> n;
};

// One iteration over the jobs in `act` (scheduler thread, mu not held).
// Returns the jobs whose computation was completed in this iteration.
hipError_t run_iteration(smooth_ctx *c, const std::vector<Job *> &act, int64_t batch,
                         std::vector<Job *> *completed, std::vector<Job *> *failed,
                         std::vector<Job *> *gs_ran) {
    hipStream_t s = c->s_comp;
    for (Job *j : act) {
        const double a = j->spec.weights.center, b = j->spec.weights.neighbor;
        hipError_t e = hipSuccess;  // this job's set-up only
        if (j->ph == PH_READY) {
            j->st.t_start_ns = now_ns();
            j->st.batch_id = (int32_t)batch;
            if (!j->refined && !j->gs) {
                e = launch_copy_ghosts(false, j->g, j->u, j->s64, s);
            } else if (j->refined && j->spec.sweeps > 0) {
                e = launch_defect(j->g, j->u, nullptr, a, b, 0.0, nullptr, j->r32, s);
                const size_t N = (size_t)j->g.count();
                if (e == hipSuccess) e = hipMemsetAsync(j->e32, 0, N * sizeof(float), s);
                if (e == hipSuccess && j->s32) e = hipMemsetAsync(j->s32, 0, N * sizeof(float), s);
            }
            if (e != hipSuccess) {
                failed->push_back(j);
                continue;
            }
            j->ph = j->spec.sweeps > 0 ? PH_PASSES : PH_FINISH;
        }
    }
    // Rounds of batched launches: every job still in its passes takes one
    // more Jacobi pass or its next block of Gauss-Seidel sweeps per round,
    // until it has done sweeps_per_iteration sweeps in this iteration (0 =
    // all of them); a job's launches follow each other on the stream.
    std::map<Job *, int> done_now;
    const int spi = c->cfg.sweeps_per_iteration;
    for (;;) {
        std::map<int, JacGroup> jg;
        std::map<int, GsGroup> gg;
        for (Job *j : act) {
            if (j->ph != PH_PASSES) continue;
            if (std::find(failed->begin(), failed->end(), j) != failed->end()) continue;
            if (spi > 0 && done_now[j] >= spi) continue;
            const double a = j->spec.weights.center, b = j->spec.weights.neighbor;
            const bool ha = a != 0.0;
            {
                const bool f32 = j->refined;
                if (!j->gs) {
                    const int tb = j->plan[j->pass];
                    const int key = (f32 ? 1000 : 0) + tb * 10 + (ha ? 2 : 0) + (f32 ? 1 : 0);
                    JacGroup &G = jg[key];
                    G.fp32 = f32;
                    G.tb = tb;
                    G.ha = ha;
                    G.hf = f32;
                    JacBatchItem it;
                    it.g = j->g;
                    if (!f32) {
                        it.src = j->parity ? (const void *)j->s64 : (const void *)j->u;
                        it.dst = j->parity ? (void *)j->u : (void *)j->s64;
                        it.f = nullptr;
                        it.gw = 0.0;
                    } else {
                        it.src = j->parity ? (const void *)j->s32 : (const void *)j->e32;
                        it.dst = j->parity ? (void *)j->e32 : (void *)j->s32;
                        it.f = j->r32;
                        it.gw = 1.0;
                    }
                    it.a = a;
                    it.b = b;
                    G.items.push_back(it);
                    G.jobs.push_back(j);
                } else {
                    const int key = 100000 + (f32 ? 10 : 0) + (ha ? 2 : 0) + (f32 ? 1 : 0);
                    GsGroup &G = gg[key];
                    G.fp32 = f32;
                    G.ha = ha;
                    G.hf = f32;
                    GsBatchItem it;
                    it.g = j->g;
                    it.u = f32 ? (void *)j->e32 : (void *)j->u;
                    it.f = f32 ? (const void *)j->r32 : nullptr;
                    it.a = a;
                    it.b = b;
                    it.gw = f32 ? 1.0 : 0.0;
                    const int left = j->spec.sweeps - j->sweeps_done;
                    it.sweeps = spi > 0 ? std::min(spi - done_now[j], left) : left;
                    G.items.push_back(it);
                    G.jobs.push_back(j);
                    G.n.push_back(it.sweeps);
                }
            }
        }
        if (jg.empty() && gg.empty()) break;
        // batched launches of this round
        for (auto &kv : jg) {
            JacGroup &G = kv.second;
            hipError_t e = hipSuccess;
            auto &tab = c->jac_tables[kv.first];
            const size_t need = jacobi_batch_table_bytes((int)G.items.size());
            if (tab.second < need) {
                if (tab.first) (void)hipFree(tab.first);
                tab.first = nullptr;
                tab.second = 0;
                e = hipMalloc(&tab.first, need * 2);
                if (e == hipSuccess) tab.second = need * 2;
            }
            if (e == hipSuccess)
                e = launch_jacobi_batch(G.fp32, G.tb, G.ha, G.hf, G.items, tab.first, G.staging, s);
            if (e != hipSuccess) {
                for (Job *j : G.jobs) failed->push_back(j);
                continue;
            }
            for (Job *j : G.jobs) {
                done_now[j] += G.tb;
                j->parity ^= 1;
                if (++j->pass == j->plan.size()) j->ph = PH_FINISH;
            }
        }
        for (auto &kv : gg) {
            GsGroup &G = kv.second;
            auto &w = c->gs_works[kv.first];
            if (!w) w.reset(new GsBatchWork());
            const hipError_t e = launch_gs_batch(G.fp32, G.ha, G.hf, G.items, *w, s);
            if (e != hipSuccess) {
                for (Job *j : G.jobs) failed->push_back(j);
                continue;
            }
            for (size_t i = 0; i < G.jobs.size(); ++i) {
                Job *j = G.jobs[i];
                if (std::find(gs_ran->begin(), gs_ran->end(), j) == gs_ran->end()) gs_ran->push_back(j);
                done_now[j] += G.n[i];
                j->sweeps_done += G.n[i];
                if (j->sweeps_done >= j->spec.sweeps) j->ph = PH_FINISH;
            }
        }
    }  // rounds
    // jobs whose sweeps are done: FP64 correction for refined jobs, then hand
    // over to the downloader
    for (Job *j : act) {
        if (j->ph != PH_FINISH) continue;
        if (std::find(failed->begin(), failed->end(), j) != failed->end()) continue;
        hipError_t e = hipSuccess;
        if (j->refined && j->spec.sweeps > 0) {
            const float *res = (!j->gs && j->parity) ? j->s32 : j->e32;
            e = launch_correct(j->g, j->u, res, true, s);
        }
        j->result = (!j->refined && !j->gs && j->parity) ? j->s64 : j->u;
        if (e == hipSuccess) e = hipEventCreateWithFlags(&j->ev_done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(j->ev_done, s);
        if (e != hipSuccess) {
            failed->push_back(j);
            continue;
        }
        j->ph = PH_DOWNLOADING;
        completed->push_back(j);
    }
    return hipSuccess;
}

void scheduler(smooth_ctx *c) {
    (void)hipSetDevice(c->cfg.device);
    std::unique_lock<std::mutex> lk(c->mu);
    for (;;) {
        admit(c);
        std::vector<Job *> act;
        for (Job *j : c->resident)
            if (j->ph == PH_READY || j->ph == PH_PASSES || j->ph == PH_FINISH) act.push_back(j);
        if (act.empty()) {
            if (c->stop && c->pending.empty() && c->resident.empty()) break;
            c->cv.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        const int64_t batch = c->batches++;
        lk.unlock();
        std::vector<Job *> completed, failed, gs_ran;
        (void)run_iteration(c, act, batch, &completed, &failed, &gs_ran);
        hipError_t e = hipEventRecord(c->ev_iter, c->s_comp);
        if (e == hipSuccess) e = hipEventSynchronize(c->ev_iter);
        if (e == hipSuccess && !gs_ran.empty()) {
            // a wavefront batch that gave up waiting leaves partial results
            uint32_t st = 0;
            e = gs_status(c->cfg.device, c->s_comp, true, &st);
            if (e == hipSuccess && (st & 1u)) {
                set_error("job iteration: a Gauss-Seidel wavefront gave up waiting");
                for (Job *j : gs_ran) failed.push_back(j);
            }
        }
        lk.lock();
        if (e != hipSuccess) {
            set_error(std::string("job iteration: ") + hipGetErrorString(e));
            for (Job *j : act)
                if (j->ph != PH_END) finish(c, j, SMOOTH_FAILED);
            continue;
        }
        for (Job *j : failed)
            if (j->ph != PH_END) finish(c, j, SMOOTH_FAILED);
        const int64_t t_iter = now_ns();
        for (Job *j : completed)
            if (j->ph != PH_END) {
                j->st.t_computed_ns = t_iter;
                c->to_download.push_back(j);
            }
        if (!completed.empty()) c->cv_io.notify_all();
    }
    c->sched_done = true;
    c->cv_io.notify_all();
}

bool terminal(int32_t s) {
    return s == SMOOTH_DONE || s == SMOOTH_FAILED || s == SMOOTH_CANCELED;
}

int fail(int status, const std::string &m) {
    set_error(m);
    return status;
}

}  // namespace

// Pass schedule shared with stencil_jacobi (api.cpp).
namespace stk {
std::vector<int> jacobi_pass_plan(bool fp32, bool rhs, int sweeps, int t_fuse, bool *final_copy);
}

extern "C" {

int smooth_init(const smooth_config *cfg, smooth_ctx **out) {
    if (!cfg || !out) return fail(ST_EINVAL, "config and out must not be NULL");
    if (cfg->max_inflight < 1) return fail(ST_EINVAL, "max_inflight must be >= 1");
    if (cfg->sweeps_per_iteration < 0)
        return fail(ST_EINVAL, "sweeps_per_iteration must be >= 0");
    if (cfg->hbm_budget_bytes < 4096) return fail(ST_EINVAL, "hbm_budget_bytes too small");
    if (!((cfg->t_fuse >= 0 && cfg->t_fuse <= 8) || cfg->t_fuse == 16))
        return fail(ST_EINVAL, "t_fuse must be 0..8 or 16");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
        return fail(ST_EINVAL, "no such HIP device");
    std::unique_ptr<smooth_ctx> c(new smooth_ctx());
    c->cfg = *cfg;
    hipError_t e = hipSetDevice(cfg->device);
    if (e == hipSuccess) e = hipMalloc(&c->pool, cfg->hbm_budget_bytes);
    if (e != hipSuccess) {
        c->pool = nullptr;
        return fail(ST_ENOMEM, std::string("job pool: ") + hipGetErrorString(e));
    }
    c->alloc.reset(cfg->hbm_budget_bytes);
    c->s_up.assign(kIoThreads, nullptr);
    c->s_down.assign(kIoThreads, nullptr);
    e = hipStreamCreateWithFlags(&c->s_comp, hipStreamNonBlocking);
    for (int k = 0; k < kIoThreads && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&c->s_up[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->s_down[k], hipStreamNonBlocking);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_iter, hipEventDisableTiming);
    if (e != hipSuccess) {
        for (hipStream_t st : c->s_up)
            if (st) (void)hipStreamDestroy(st);
        for (hipStream_t st : c->s_down)
            if (st) (void)hipStreamDestroy(st);
        if (c->s_comp) (void)hipStreamDestroy(c->s_comp);
        (void)hipFree(c->pool);
        return fail(ST_EHIP, std::string("job service streams: ") + hipGetErrorString(e));
    }
    smooth_ctx *p = c.release();
    p->th_sched = std::thread(scheduler, p);
    for (int k = 0; k < kIoThreads; ++k) {
        p->th_up.emplace_back(uploader, p, k);
        p->th_down.emplace_back(downloader, p, k);
    }
    *out = p;
    return ST_OK;
}

int smooth_submit(smooth_ctx *c, const smooth_job *job, uint64_t *job_id) {
    if (!c || !job || !job_id) return fail(ST_EINVAL, "ctx, job and job_id must not be NULL");
    if (job->nx < 1 || job->ny < 1 || job->nz < 1) return fail(ST_EINVAL, "extents must be >= 1");
    if (job->method != SMOOTH_JACOBI && job->method != SMOOTH_GS)
        return fail(ST_EINVAL, "method must be SMOOTH_JACOBI or SMOOTH_GS");
    if (job->precision != SMOOTH_FP64 && job->precision != SMOOTH_FP32_REFINED)
        return fail(ST_EINVAL, "precision must be SMOOTH_FP64 or SMOOTH_FP32_REFINED");
    if (job->sweeps < 0) return fail(ST_EINVAL, "sweeps must be >= 0");
    if (!job->input_host || !job->output_host)
        return fail(ST_EINVAL, "input_host and output_host must not be NULL");
    const int64_t px = job->nx + 2, py = job->ny + 2, pz = job->nz + 2;
    if (px * py >= ((int64_t)1 << 28) || pz >= ((int64_t)1 << 31))
        return fail(ST_EINVAL, "grid too large (one padded plane must hold < 2^28 elements)");
    if (job->method == SMOOTH_GS && (job->ny > 8192 || job->nz > 8192))
        return fail(ST_EINVAL, "Gauss-Seidel supports ny, nz <= 8192");
    std::unique_ptr<Job> j(new Job());
    j->spec = *job;
    j->gs = job->method == SMOOTH_GS;
    j->refined = job->precision == SMOOTH_FP32_REFINED;
    j->g.nx = (int)job->nx;
    j->g.ny = (int)job->ny;
    j->g.nz = (int)job->nz;
    j->g.h = 1;
    j->g.px = px;
    j->g.py = py;
    j->g.pz = pz;
    j->bytes = footprint(*job);
    j->st.lups = (double)job->nx * job->ny * job->nz * job->sweeps;
    if (!j->gs && job->sweeps > 0) {
        bool fc = false;
        j->plan = jacobi_pass_plan(j->refined, j->refined, job->sweeps, c->cfg.t_fuse, &fc);
    }
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->stop) return fail(ST_EBUSY, "service is shutting down");
    if (PoolAllocator::round_up(j->bytes) > c->alloc.size())
        return fail(ST_EINVAL, "job footprint exceeds the HBM budget");
    j->id = c->next_id++;
    j->st.t_submit_ns = now_ns();
    *job_id = j->id;
    c->pending.push_back(j.get());
    c->jobs[j->id] = std::move(j);
    c->cv.notify_all();
    return ST_OK;
}

int smooth_poll(smooth_ctx *c, uint64_t job_id, int32_t *state, smooth_stats *stats) {
    if (!c || !state) return fail(ST_EINVAL, "ctx and state must not be NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    auto it = c->jobs.find(job_id);
    if (it == c->jobs.end()) return fail(ST_ENOENT, "unknown job id");
    *state = it->second->state;
    if (stats) *stats = it->second->st;
    return ST_OK;
}

int smooth_wait_all(smooth_ctx *c, int64_t timeout_ms) {
    if (!c) return fail(ST_EINVAL, "ctx is NULL");
    std::unique_lock<std::mutex> lk(c->mu);
    auto all_done = [&] {
        for (auto &kv : c->jobs)
            if (!terminal(kv.second->state)) return false;
        return true;
    };
    if (timeout_ms < 0) {
        c->cv_done.wait(lk, all_done);
        return ST_OK;
    }
    if (!c->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), all_done))
        return fail(ST_EBUSY, "jobs still running at timeout");
    return ST_OK;
}

int smooth_service_info(smooth_ctx *c, smooth_service_stats *out) {
    if (!c || !out) return fail(ST_EINVAL, "ctx and out must not be NULL");
    std::lock_guard<std::mutex> lk(c->mu);
    out->pool_bytes = c->alloc.size();
    out->footprint_high_water = c->alloc.high_water();
    out->footprint_now = c->alloc.used();
    out->batches = c->batches;
    out->jobs_done = c->n_done;
    out->jobs_failed = c->n_failed;
    out->jobs_canceled = c->n_canceled;
    out->max_resident_seen = c->max_resident;
    out->reserved = 0;
    return ST_OK;
}

int smooth_shutdown(smooth_ctx *c) {
    if (!c) return fail(ST_EINVAL, "ctx is NULL");
    {
        std::lock_guard<std::mutex> lk(c->mu);
        c->stop = true;
        while (!c->pending.empty()) {
            Job *j = c->pending.front();
            c->pending.pop_front();
            finish(c, j, SMOOTH_CANCELED);
        }
        c->cv.notify_all();
        c->cv_io.notify_all();
    }
    if (c->th_sched.joinable()) c->th_sched.join();
    for (auto &t : c->th_up)
        if (t.joinable()) t.join();
    for (auto &t : c->th_down)
        if (t.joinable()) t.join();
    (void)hipSetDevice(c->cfg.device);
    (void)hipDeviceSynchronize();
    for (auto &kv : c->jac_tables)
        if (kv.second.first) (void)hipFree(kv.second.first);
    c->gs_works.clear();
    if (c->ev_iter) (void)hipEventDestroy(c->ev_iter);
    if (c->s_comp) (void)hipStreamDestroy(c->s_comp);
    for (hipStream_t st : c->s_up)
        if (st) (void)hipStreamDestroy(st);
    for (hipStream_t st : c->s_down)
        if (st) (void)hipStreamDestroy(st);
    if (c->pool) (void)hipFree(c->pool);
    delete c;
    return ST_OK;
}

}  // extern "C"
