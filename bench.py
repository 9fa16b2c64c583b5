#!/usr/bin/env python3
"""Benchmark of the iterated 3D 7-point smoothers on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--quick] [--no-cpu]

One *step* is the headline workload: 100 FP64 Jacobi sweeps on a 512^3
interior (ghost and interior values U[0,1), a = 0, b = 1/6), fused t sweeps
per pass over HBM (t chosen by the library unless --t is given).  The value is
MLUP/s = 512^3 * 100 * K / (time of K steps); inputs are resident in HBM
before the timed region.  Defaults: K = 20 timed steps after W = 10 untimed
ones (about 0.1 s of warm-up, enough for the clocks to settle).  Extra fields report every t, FP32 storage, the
Gauss-Seidel wavefront on 384^3 x 50, the FP32-refined vs plain FP64 Poisson
solve, and the serving stream, each measured after the headline.

The roofline object prices the dominant kernel (the fused Jacobi pass) against
8 TB/s: algorithmic bytes per pass = 2 * sizeof(double) * 512^3 (one load and
one store per site, Eq. (1) of the paper divided over t fused sweeps).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
SECTIONS = ("copy", "small", "by_t", "fp32", "gs", "gs512", "rbgs", "mg", "poisson", "serving")


def gs_source_sha():
    """Hash of the Gauss-Seidel wavefront source (comments and blank lines
    removed), as recorded in its counter profile."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_1004_1741_amd", "csrc", "gs.hip")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in src.split("\n")]
    return hashlib.sha256("\n".join(ln for ln in lines if ln.strip()).encode()).hexdigest()[:16]


def measured_gs_traffic(n):
    """HBM bytes per launch of the wavefront (50 sweeps at n^3) from the
    committed counter summary, or None if it describes other sources."""
    prof = os.path.join(ROOT, "profiles", "gs_wavefront_fp64_%dcubed.md" % n)
    if not os.path.exists(prof):
        return None
    vals = {}
    for line in open(prof):
        if " = " in line:
            k, v = line.strip().split(" = ", 1)
            vals[k] = v
    if vals.get("kernel_source_sha256_16") != gs_source_sha():
        return None
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except KeyError:
        return None


def bytes_per_lup(elem_bytes: int, t: int) -> float:
    """Eq. (1): one load and one store per site per pass of t fused sweeps."""
    return 2.0 * elem_bytes / t


def eq1_mlups(bandwidth_GBs: float, elem_bytes: int = 8, t: int = 1) -> float:
    """Bandwidth-bound lattice-site updates per second, Eq. (1), in MLUP/s."""
    return bandwidth_GBs * 1e9 / bytes_per_lup(elem_bytes, t) / 1e6


def jacobi_source_sha(t):
    """Hash of the fused-pass kernel source as built for depth t, with
    comments and blank lines removed (a comment edit does not change the
    kernel the counters describe)."""
    import hashlib
    import re
    cs = os.path.join(ROOT, "paper_1004_1741_amd", "csrc")
    h = hashlib.sha256()
    for name in ("jacobi_impl.h", "jacobi_t%d.hip" % t):
        src = open(os.path.join(cs, name)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in src.split("\n")]
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_t, n):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, each scaled by the
    plain-copy calibration), or None if that summary does not describe the
    kernel as it is now built (source changed) or this workload."""
    prof = os.path.join(ROOT, "profiles", "jacobi_pass_fp64_t%d_512cubed.md" % kernel_t)
    if n != 512 or not os.path.exists(prof):
        return None
    vals = {}
    for line in open(prof):
        if " = " in line:
            k, v = line.strip().split(" = ", 1)
            vals[k] = v
    if vals.get("kernel_source_sha256_16") != jacobi_source_sha(kernel_t):
        return None
    return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--sweeps", type=int, default=100)
    ap.add_argument("--t", type=int, default=0, help="fused sweeps per pass (0 = library choice)")
    ap.add_argument("--quick", action="store_true", help="headline only (same as --sections none)")
    ap.add_argument("--sections", default="all",
                    help="extra measurements after the headline, comma separated: "
                         "copy,small,by_t,fp32,gs,gs512,rbgs,mg,poisson,serving (or all / none)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--poisson-n", type=int, default=512)
    ap.add_argument("--poisson-m", type=int, default=32, help="inner sweeps per outer round")
    ap.add_argument("--poisson-methods", default="rbgs",
                    help="smoothers of the large Poisson comparison (jacobi,gs,rbgs)")
    ap.add_argument("--poisson-inner", default="fp32_refined,plain_fp64",
                    help="which solves of the Poisson comparison to run")
    ap.add_argument("--serving-jobs", type=int, default=2000)
    ap.add_argument("--serving-rate", default="50,100,200,500",
                    help="arrival rate(s) per second, comma separated")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 2 GiB device copy (counter calibration)")
    return ap.parse_args()


def events_time(torch, fn, reps=1):
    """Time fn() reps times on the current stream with HIP events (ms)."""
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1)


def copy_bandwidth(torch, nbytes=2 << 30):
    """Achievable HBM bandwidth of a plain device copy (GB/s, read + write)."""
    n = nbytes // 8
    a = torch.empty(n, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    ms = events_time(torch, lambda: b.copy_(a), reps=10) / 10
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def jacobi_run(P, torch, u, s, sweeps, t):
    P.jacobi(u, s, sweeps, a=0.0, b=1.0 / 6.0, t_fuse=t)


def cpu_baseline(n, target_s=15.0):
    """The CPU oracle (single thread, as it stands) on a bounded sample."""
    import oracle
    import synthetic_inputs as si
    lib = oracle.load()
    u = si.jacobi_512(seed=0, n=n)["u"]
    # one untimed sweep (first-touch of the buffers); the per-sweep cost is
    # the difference of a 3-sweep and a 1-sweep call (each call also copies
    # and allocates), then enough sweeps for ~target_s seconds
    oracle.jacobi(u, 1, lib=lib)
    t0 = time.perf_counter()
    oracle.jacobi(u, 1, lib=lib)
    t1 = time.perf_counter()
    oracle.jacobi(u, 3, lib=lib)
    t3 = time.perf_counter()
    one = max((t3 - t1) - (t1 - t0), 1e-3) / 2
    S = max(1, min(100, int(round(target_s / one))))
    t0 = time.perf_counter()
    oracle.jacobi(u, S, lib=lib)
    dt = time.perf_counter() - t0
    lups = float(n) ** 3 * S
    return {"value": lups / dt / 1e6, "unit": "MLUP/s", "cores": 1, "kind": "oracle",
            "sample": "FP64 Jacobi %d^3 x %d sweeps (of the 100-sweep step), single-threaded "
                      "C oracle, %.1f s" % (n, S, dt)}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_threads_baseline(n, target_s=10.0):
    """The oracle's Jacobi loops with the k loop on all OpenMP threads the
    process may use (OMP_NUM_THREADS, else every core): a CPU Jacobi
    baseline next to the single-threaded oracle."""
    import oracle
    import synthetic_inputs as si
    lib = oracle.load()
    u = si.jacobi_512(seed=0, n=n)["u"]
    oracle.jacobi_threads(u, 1, lib=lib)
    t0 = time.perf_counter()
    oracle.jacobi_threads(u, 1, lib=lib)
    t1 = time.perf_counter()
    oracle.jacobi_threads(u, 3, lib=lib)
    t3 = time.perf_counter()
    one = max((t3 - t1) - (t1 - t0), 1e-3) / 2
    S = max(1, min(100, int(round(target_s / one))))
    t0 = time.perf_counter()
    _, used = oracle.jacobi_threads(u, S, lib=lib)
    dt = time.perf_counter() - t0
    return {"value": round(float(n) ** 3 * S / dt / 1e6, 1), "unit": "MLUP/s", "cores": used,
            "kind": "oracle loops, OpenMP over k",
            "sample": "FP64 Jacobi %d^3 x %d sweeps, %d threads, %.1f s" % (n, S, used, dt)}


def cpu_refine_oracle(ns=(32, 64), m=32, tol=1e-10):
    """The oracle's defect-correction solve (FP64 throughout, and with float
    inner sweeps) to rel <= tol on the Poisson workload at small n, single
    thread: the CPU side of the solve comparison."""
    import oracle
    import synthetic_inputs as si
    lib = oracle.load()
    out = {}
    for n in ns:
        w = si.poisson(n=n, seed=0)
        fp = w["f"] / float((n + 1) ** 2)
        for method, name in ((0, "jacobi"), (1, "gauss_seidel")):
            # the oracle's FP64 variant is the same defect correction with FP64
            # inner sweeps (the GPU's plain_fp64 smooths u itself)
            for inner_f32, key in ((True, "fp32_refined"), (False, "fp64_defect_correction")):
                t0 = time.perf_counter()
                _, rc, outer, rel = oracle.refine(w["u"], fp, method=method, inner_f32=inner_f32,
                                                  m=m, tol=tol, max_outer=10 ** 6, lib=lib)
                dt = time.perf_counter() - t0
                out["%d_%s_%s" % (n, name, key)] = {
                    "seconds": round(dt, 3), "outer_rounds": outer, "sweeps": outer * m,
                    "rel_residual": rel, "status": rc,
                    "MLUPs": round(float(n) ** 3 * outer * m / dt / 1e6, 1)}
                log("cpu oracle refine %d^3 %s %s: %s" % (n, name, key, out["%d_%s_%s" % (n, name, key)]))
    return out


def cpu_gs_oracle(n=384, sweeps=50):
    """The CPU oracle's lexicographic Gauss-Seidel (inherently sequential,
    single thread) on the full 384^3 x 50 workload."""
    import oracle
    import synthetic_inputs as si
    lib = oracle.load()
    g = si.gs_384(seed=0, n=n)
    oracle.gauss_seidel(g["u"], 1, lib=lib)  # first touch
    t0 = time.perf_counter()
    oracle.gauss_seidel(g["u"], sweeps, lib=lib)
    dt = time.perf_counter() - t0
    return {"value": round(float(n) ** 3 * sweeps / dt / 1e6, 1), "unit": "MLUP/s", "cores": 1,
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": "FP64 Gauss-Seidel %d^3 x %d sweeps, single-threaded C oracle" % (n, sweeps)}


def small_grids(P, torch):
    """The 64^3 x 10 smoke configuration: grids of 2.3 MB stay in L2/MALL, so
    these rates are cache-resident and launch/latency-bound, not HBM numbers."""
    import synthetic_inputs as si
    w = si.jacobi_small(seed=0)
    u = torch.from_numpy(w["u"]).to("cuda")
    s = torch.empty_like(u)
    S = w["sweeps"]
    lups = 64.0 ** 3 * S
    out = {"label": "cache-resident"}
    P.jacobi(u, s, S, a=w["a"], b=w["b"])
    ms = events_time(torch, lambda: P.jacobi(u, s, S, a=w["a"], b=w["b"]), reps=20) / 20
    out["jacobi_fp64_64cubed_x10"] = {"ms": round(ms, 4), "MLUPs": round(lups / (ms * 1e-3) / 1e6)}
    g = si.gs_384(seed=0, n=64)
    ug = torch.from_numpy(g["u"]).to("cuda")
    P.gauss_seidel(ug, S)
    ms = events_time(torch, lambda: P.gauss_seidel(ug, S), reps=20) / 20
    out["gs_fp64_64cubed_x10"] = {"ms": round(ms, 4), "MLUPs": round(lups / (ms * 1e-3) / 1e6)}
    log("small grids: %s" % out)
    return out


def mg_solves(P, torch, n, keep, seed=0, tol=1e-10):
    """The Poisson workload solved by multigrid V(2,2)-cycles inside FP64
    defect correction: every smoother, FP32 and FP64 cycles; time to
    rel <= tol.  The FP32 red-black solution is kept for the CPU residual
    check."""
    import synthetic_inputs as si
    w = si.poisson(n=n, seed=seed)
    fp_host = w["f"] / float((n + 1) ** 2)
    fp = torch.from_numpy(fp_host).to("cuda")
    out = {}
    for sm, name in ((2, "red_black"), (1, "gauss_seidel"), (0, "weighted_jacobi")):
        for fp32, key in ((True, "fp32_cycles"), (False, "fp64_cycles")):
            u = torch.from_numpy(w["u"]).to("cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            cyc, rel, rc = P.mg_solve(u, fp, smoother=sm, inner_fp32=fp32, pre=2, post=2,
                                      rel_tol=tol, max_cycles=100, raise_on_noconv=False)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            out["%s_%s" % (name, key)] = {"seconds": round(dt, 4), "cycles": cyc,
                                          "rel_residual": rel, "status": rc,
                                          "ms_per_cycle": round(1e3 * dt / max(cyc, 1), 2)}
            log("mg %d^3 %s %s: %s" % (n, name, key, out["%s_%s" % (name, key)]))
            if sm == 2 and fp32:
                keep["mg_%d_red_black_fp32_cycles" % n] = (u.cpu().numpy(), fp_host)
            del u
    return out


def cpu_residual_check(solutions):
    """The CPU oracle's own residual ||f' - A u|| / ||f'|| of GPU solutions."""
    import oracle
    lib = oracle.load()
    out = {}
    for key, (u, fp) in solutions.items():
        t0 = time.perf_counter()
        _, rr = oracle.residual(u, fp, lib=lib)
        rel = float(np.sqrt(rr) / np.sqrt(oracle.sumsq(fp, lib=lib)))
        out[key] = {"rel_residual": rel, "seconds": round(time.perf_counter() - t0, 2)}
    return out


def cpu_wavefront(n, gs_n=384, sweeps=8):
    """The paper's own multicore schemes on the host cores (cpu_baseline/):
    the threaded Jacobi baseline (t = 1) and the temporal wavefront (t = 4, 8)
    on n^3, the pipeline-parallel Gauss-Seidel (t = 1) and its wavefront
    (t = 4) on gs_n^3, `sweeps` sweeps each, FP64."""
    import cpu_baseline as W
    import synthetic_inputs as si
    W.build(force=False)
    threads = min(W.cpu_count(), int(os.environ.get("OMP_NUM_THREADS", "16") or 16), 64)
    out = {"threads": threads, "host": cpu_model()}
    u = si.jacobi_512(seed=0, n=n)["u"]
    scratch = np.empty_like(u)
    for t in (1, 4, 8):
        groups = max(1, threads // t)
        if t > threads:
            continue
        by = max(16, n // (2 * groups))  # two y-blocks per group: contiguous rows per plane
        W.jacobi(u, t, t=t, groups=groups, block_y=by, scratch=scratch)  # first touch
        t0 = time.perf_counter()
        W.jacobi(u, sweeps, t=t, groups=groups, block_y=by, scratch=scratch)
        dt = time.perf_counter() - t0
        out["jacobi_%d_t%d" % (n, t)] = {"MLUPs": round(float(n) ** 3 * sweeps / dt / 1e6, 1),
                                         "threads": t * groups, "groups": groups,
                                         "block_rows": by, "seconds": round(dt, 3)}
    del u, scratch
    g = si.gs_384(seed=0, n=gs_n)["u"]
    for t in (1, 4):
        P_ = max(1, threads // t)
        t0 = time.perf_counter()
        W.gauss_seidel(g, sweeps, t=t, subblocks=P_)
        dt = time.perf_counter() - t0
        out["gs_%d_t%d" % (gs_n, t)] = {"MLUPs": round(float(gs_n) ** 3 * sweeps / dt / 1e6, 1),
                                        "threads": t * P_, "subblocks": P_,
                                        "seconds": round(dt, 3)}
    return out


def poisson_compare(P, torch, n, seed=0, methods=(0, 1, 2), m=32, tol=1e-10, chunk_s=30.0,
                    inners=("fp32_refined", "plain_fp64"), keep=None):
    """-Laplace u = f on n^3, h = 1/(n+1), f U[-1,1), u0 = 0: time to reach
    ||f' - A u|| <= tol ||f'|| with the FP32-refined loop and the plain FP64
    method.  The solve runs as consecutive library calls of a bounded number
    of outer rounds (each call continues from the current u and re-checks the
    residual first, so the iterates are those of one uninterrupted solve),
    with a progress line after each call."""
    import synthetic_inputs as si
    w = si.poisson(n=n, seed=seed)
    fp = torch.from_numpy(w["f"] / float((n + 1) ** 2)).to("cuda")
    out = {}
    for method in methods:
        name = ("jacobi", "gauss_seidel", "red_black")[method]
        res = {}
        for inner_fp32, key in ((True, "fp32_refined"), (False, "plain_fp64")):
            if key not in inners:
                continue
            u = torch.from_numpy(w["u"]).to("cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rounds, rel, rc, per_call = 0, 1.0, -6, 16
            while True:
                t1 = time.perf_counter()
                r, rel, rc = P.refine_solve(u, fp, method=method, inner_fp32=inner_fp32,
                                            inner_sweeps=m, rel_tol=tol, max_outer=per_call,
                                            raise_on_noconv=False)
                torch.cuda.synchronize()
                rounds += r
                dt_call = time.perf_counter() - t1
                log("poisson %d^3 %s %s: %d rounds, rel %.3e, %.1f s" %
                    (n, name, key, rounds, rel, time.perf_counter() - t0))
                if rc == 0 or rounds >= 10 ** 7:
                    break
                # size the next call for about chunk_s seconds
                per_call = max(1, min(10 ** 6, int(per_call * chunk_s / max(dt_call, 1e-3))))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            sweeps = rounds * m
            res[key] = {"seconds": round(dt, 3), "outer_rounds": rounds, "sweeps": sweeps,
                        "rel_residual": rel, "status": rc,
                        "MLUPs": round(float(n) ** 3 * sweeps / dt / 1e6)}
            res[key + "_u"] = u
            if keep is not None:
                keep["poisson_%d_%s_%s" % (n, name, key)] = (u.cpu().numpy(),
                                                              fp.cpu().numpy())
            log("poisson %d^3 %s %s: %s" % (n, name, key, {k: v for k, v in res[key].items()}))
        if "fp32_refined_u" in res and "plain_fp64_u" in res:
            a, b = res.pop("fp32_refined_u"), res.pop("plain_fp64_u")
            res["rel_diff_fp32_refined_vs_fp64"] = float((a - b).abs().max() / b.abs().max())
            res["speedup_fp32_refined"] = round(res["plain_fp64"]["seconds"] /
                                                res["fp32_refined"]["seconds"], 3)
            del a, b
        for k in [k for k in res if k.endswith("_u")]:
            del res[k]
        out[name] = res
    return out


def serving_streams(P, n_jobs, rates, seed=0, budget=32 << 30, max_inflight=64, keep=(),
                    sweeps_per_iteration=0):
    """Continuous-batching service under Poisson arrival streams of uneven jobs
    (extents U{32..256}, Jacobi/GS and FP64/FP32-refined 50/50, 2..20 sweeps;
    the same jobs at every rate, arrival times scaled by 1/rate).  Inputs are
    generated once, before any clock starts.  Returns one record per rate and
    the outputs of the jobs listed in `keep` (from the first rate)."""
    import threading
    from concurrent.futures import ThreadPoolExecutor
    import synthetic_inputs as si
    jobs0 = si.serving_stream(n_jobs=n_jobs, rate_per_s=rates[0], seed=seed)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        inputs = list(ex.map(lambda jb: jb.make_input(), jobs0))
    log("serving: %d job inputs generated in %.1f s (%.1f GB)" %
        (n_jobs, time.perf_counter() - t0, sum(x.nbytes for x in inputs) / 1e9))
    # Result buffers: a client reuses resident, already-faulted buffers, so a
    # pool of npool buffers of the largest job size is touched once here and
    # handed out round-robin; a buffer is reused only after the job that last
    # used it has ended (DONE, FAILED or CANCELED: the feeder waits for that,
    # and counts the waits).  The
    # jobs in `keep` get buffers of their own.
    npool = 96
    maxn = max(x.size for x in inputs)

    def touched(nelem):
        b = np.empty(nelem)
        b[::512] = 0.0
        return b

    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1))) as ex:
        pool = list(ex.map(touched, [maxn] * npool))
    runs, kept = [], {}
    for ri, rate in enumerate(rates):
        jobs = si.serving_stream(n_jobs=n_jobs, rate_per_s=rate, seed=seed)
        outputs = [None] * n_jobs
        owner = [None] * npool
        waits = [0]
        svc = P.SmoothService(budget, max_inflight=max_inflight,
                              sweeps_per_iteration=sweeps_per_iteration)
        ids = [None] * n_jobs
        t0 = time.perf_counter()

        def feeder():
            for k, jb in enumerate(jobs):
                dt = jb.arrival_s - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
                if k in keep and ri == 0:
                    outputs[k] = np.empty_like(inputs[k])
                else:
                    slot = k % npool
                    prev = owner[slot]
                    while prev is not None and svc.poll(ids[prev])[0] < P.SmoothService.DONE:
                        waits[0] += 1
                        time.sleep(1e-4)
                    owner[slot] = k
                    outputs[k] = pool[slot][:inputs[k].size].reshape(inputs[k].shape)
                ids[k] = svc.submit(inputs[k], outputs[k], jb.sweeps, method=jb.method,
                                    precision=jb.precision)

        th = threading.Thread(target=feeder)
        th.start()
        th.join()
        svc.wait_all()
        wall = time.perf_counter() - t0
        lat, parts, lups = [], {"queue": [], "upload": [], "compute": [], "download": []}, 0.0
        for k in range(n_jobs):
            st, stt = svc.poll(ids[k])
            assert st == P.SmoothService.DONE
            lat.append((stt.t_done_ns - stt.t_submit_ns) * 1e-6)
            parts["queue"].append((stt.t_admit_ns - stt.t_submit_ns) * 1e-6)
            parts["upload"].append((stt.t_uploaded_ns - stt.t_admit_ns) * 1e-6)
            parts["compute"].append((stt.t_computed_ns - stt.t_uploaded_ns) * 1e-6)
            parts["download"].append((stt.t_done_ns - stt.t_computed_ns) * 1e-6)
            lups += stt.lups
        info = svc.info()
        svc.shutdown()
        if ri == 0:
            kept = {k: outputs[k] for k in keep}
        del outputs
        lat = np.array(lat)
        rec = {"jobs": n_jobs, "rate_per_s": rate, "wall_s": round(wall, 3),
               "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3),
               "breakdown_ms": {name: {"mean": round(float(np.mean(v)), 3),
                                       "p50": round(float(np.percentile(v, 50)), 3),
                                       "p99": round(float(np.percentile(v, 99)), 3)}
                                for name, v in parts.items()},
               "MLUPs_aggregate": round(lups / wall / 1e6),
               "batches": info.batches, "max_resident": info.max_resident_seen,
               "footprint_high_water_GB": round(info.footprint_high_water / 1e9, 3),
               "budget_GB": round(budget / 1e9, 3), "result_buffer_waits": waits[0]}
        runs.append(rec)
        log("serving: %s" % rec)
    return runs, jobs0, inputs, kept


def cpu_check_serving(jobs, inputs, outputs):
    """The CPU oracle on a sample of service jobs: FP64 jobs must match it bit
    for bit, FP32-refined jobs the oracle's emulation of the same steps bit
    for bit and the FP64 result within 1e-5 of max |u|."""
    import oracle
    lib = oracle.load()
    out = {"jobs": len(outputs), "fp64_bit_exact": 0, "fp32_refined_bit_exact": 0,
           "fp32_refined_max_rel_err": 0.0}
    t0 = time.perf_counter()
    for k, got in outputs.items():
        jb = jobs[k]
        u0 = inputs[k]
        ref64 = oracle.smooth(jb.method, u0, jb.sweeps, lib=lib)
        if jb.precision == 0:
            assert np.array_equal(got, ref64), ("service job %d differs from the oracle" % k)
            out["fp64_bit_exact"] += 1
        else:
            emu = oracle.refined_job(jb.method, u0, jb.sweeps, lib=lib)
            assert np.array_equal(got, emu), ("service job %d differs from the oracle" % k)
            err = float(np.abs(got - ref64).max() / np.abs(ref64).max())
            assert err <= 1e-5, (k, err)
            out["fp32_refined_bit_exact"] += 1
            out["fp32_refined_max_rel_err"] = max(out["fp32_refined_max_rel_err"], err)
    out["seconds"] = round(time.perf_counter() - t0, 2)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (--gpus %d "
              "requested); run with --gpus 1" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    import paper_1004_1741_amd as P
    import synthetic_inputs as si

    P.lib()
    n, S = args.n, args.sweeps
    lups_step = float(n) ** 3 * S
    w = si.jacobi_512(seed=0, n=n)
    u = torch.from_numpy(w["u"]).to("cuda")
    s = torch.empty_like(u)
    del w
    log("device:", torch.cuda.get_device_name(0))

    plan, fcopy = P.jacobi_plan(S, args.t)
    passes = len(plan)

    for _ in range(args.warmup):
        jacobi_run(P, torch, u, s, S, args.t)
    torch.cuda.synchronize()
    ms = events_time(torch, lambda: jacobi_run(P, torch, u, s, S, args.t), reps=args.steps)
    ms_step = ms / args.steps
    value = lups_step / (ms_step * 1e-3) / 1e6
    log("headline: %.3f ms/step, %.0f MLUP/s, plan %s" % (ms_step, value, plan))

    # Dominant kernel: the fused pass of depth tdom.  Its average launch
    # duration is measured with HIP events over launches of that kernel only
    # (a schedule of 2*k passes of depth tdom), on the stream it runs on.
    tdom = max(plan)
    k = 12
    jacobi_run(P, torch, u, s, 2 * k * tdom, tdom)
    dom_ms = events_time(torch, lambda: jacobi_run(P, torch, u, s, 2 * k * tdom, tdom),
                         reps=2) / (2 * 2 * k)
    pass_bytes = 2 * 8 * float(n) ** 3
    achieved = pass_bytes / (dom_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(tdom, n),
            "traffic_unit": "bytes/launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)",
            "kernel": "jacobi_pass_kernel<double,t=%d>" % tdom,
            "launch_us": round(dom_ms * 1e3, 2), "algorithmic_bytes_per_launch": pass_bytes,
            "bytes_per_lup": round(bytes_per_lup(8, tdom), 3),
            "sweeps_per_launch": tdom,
            "roofline_MLUPs_at_peak": round(eq1_mlups(HBM_PEAK_GBS, 8, tdom))}
    log("dominant kernel t=%d: %.1f us/launch, %.1f GB/s" % (tdom, dom_ms * 1e3, achieved))
    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    extra = {}
    sections = set() if args.quick or args.sections == "none" else (
        set(SECTIONS) if args.sections == "all" else set(args.sections.split(",")))
    unknown = sections - set(SECTIONS)
    if unknown:
        print("unknown sections: %s" % ",".join(sorted(unknown)), file=sys.stderr)
        sys.exit(2)
    if "copy" in sections:
        extra["copy_GBs"] = round(copy_bandwidth(torch), 1)
    if "small" in sections:
        extra["small_64cubed"] = small_grids(P, torch)
    if "by_t" in sections:
        per_t = {}
        for t in (1, 2, 3, 4, 5, 6, 7, 8, 16):
            pl, _ = P.jacobi_plan(S, t)
            jacobi_run(P, torch, u, s, S, t)
            m = events_time(torch, lambda: jacobi_run(P, torch, u, s, S, t), reps=2) / 2
            pms = m / len(pl)
            per_t[str(t)] = {"ms": round(m, 3), "MLUPs": round(lups_step / (m * 1e-3) / 1e6),
                             "passes": len(pl), "pass_us": round(pms * 1e3, 1),
                             "pass_GBs": round(pass_bytes / (pms * 1e-3) / 1e9, 1),
                             "pass_frac": round(pass_bytes / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            log("jacobi fp64 t=%d: %s" % (t, per_t[str(t)]))
        extra["jacobi_fp64_by_t"] = per_t
        extra["speedup_best_vs_t1"] = round(
            max(v["MLUPs"] for v in per_t.values()) / per_t["1"]["MLUPs"], 2)
    if "fp32" in sections:
        # FP32 storage
        u32 = u.float()
        s32 = torch.empty_like(u32)
        per32 = {}
        for t in (1, 2, 3, 4, 5, 6, 7, 8):
            jacobi_run(P, torch, u32, s32, S, t)
            m = events_time(torch, lambda: jacobi_run(P, torch, u32, s32, S, t), reps=2) / 2
            pl, _ = P.jacobi_plan(S, t, fp32=True)
            pms = m / len(pl)
            pb32 = pass_bytes / 2  # 4-byte elements: one load and one store per site
            per32[str(t)] = {"ms": round(m, 3), "MLUPs": round(lups_step / (m * 1e-3) / 1e6),
                             "passes": len(pl), "pass_us": round(pms * 1e3, 1),
                             "pass_GBs": round(pb32 / (pms * 1e-3) / 1e9, 1),
                             "pass_frac": round(pb32 / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            log("jacobi fp32 t=%d: %s" % (t, per32[str(t)]))
        extra["jacobi_fp32_by_t"] = per32
        del u32, s32
    if "gs" in sections:
        # Gauss-Seidel wavefront, 384^3 x 50
        g = si.gs_384(seed=0)
        ug = torch.from_numpy(g["u"]).to("cuda")
        gl = 384.0 ** 3 * g["sweeps"]
        gs = {}
        for t in (0, 1):
            u0 = ug.clone()
            P.gauss_seidel(u0, g["sweeps"], t_fuse=t)
            u0.copy_(ug)
            m = events_time(torch, lambda: P.gauss_seidel(u0, g["sweeps"], t_fuse=t), reps=1)
            key = "all_sweeps_in_flight" if t == 0 else "one_launch_per_sweep"
            # algorithmic HBM bytes: one load and one store per site per launch
            launches = 1 if t == 0 else g["sweeps"]
            gbytes = 2 * 8 * 384.0 ** 3 * launches
            gs[key] = {"ms": round(m, 3), "MLUPs": round(gl / (m * 1e-3) / 1e6),
                       "hbm_bytes_algorithmic": gbytes,
                       "hbm_frac": round(gbytes / (m * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            log("gs 384^3 x50 %s: %s" % (key, gs[key]))
        extra["gs_384_x50"] = gs
        del ug, u0
    if "gs512" in sections:
        # Gauss-Seidel wavefront at the headline size: 512^3 x 50, all sweeps
        # in flight (interior 2U-1 seed 0, zero ghosts)
        g = si.gs_384(seed=0, n=n)
        ug = torch.from_numpy(g["u"]).to("cuda")
        u0 = ug.clone()
        P.gauss_seidel(u0, 50)
        P.sync()
        u0.copy_(ug)
        m = events_time(torch, lambda: P.gauss_seidel(u0, 50), reps=1)
        P.sync()
        gbytes = 2 * 8 * float(n) ** 3
        gl = float(n) ** 3 * 50
        t1_ms = 50 * gbytes / (HBM_PEAK_GBS * 1e9) * 1e3  # one load + store per site per sweep
        extra["gs_%d_x50" % n] = {
            "ms": round(m, 3), "MLUPs": round(gl / (m * 1e-3) / 1e6),
            "frac_of_t1_roofline": round(t1_ms / m, 4),
            "hbm_bytes_algorithmic": gbytes,
            "hbm_frac": round(gbytes / (m * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
            "traffic": measured_gs_traffic(n),
            "traffic_unit": "bytes/launch (rocprofv3 FETCH_SIZE+WRITE_SIZE, copy-calibrated)"}
        log("gs %d^3 x50: %s" % (n, extra["gs_%d_x50" % n]))
        del ug, u0
    if "rbgs" in sections:
        # red-black Gauss-Seidel on the fused pass, 512^3 x 100 sweeps (FP64)
        rb = {}
        for t in (0, 1, 2, 3, 4):
            jacobi_run_rb = lambda: P.red_black(u, s, S, t_fuse=t)
            jacobi_run_rb()
            m = events_time(torch, jacobi_run_rb, reps=2) / 2
            rb[str(t)] = {"ms": round(m, 3), "MLUPs": round(lups_step / (m * 1e-3) / 1e6)}
            log("red-black fp64 512^3 x%d t=%d: %s" % (S, t, rb[str(t)]))
        extra["rbgs_fp64_512_x100_by_t"] = rb
    torch.cuda.synchronize()
    # free the 512^3 grids before the remaining measurements
    del u, s
    torch.cuda.empty_cache()
    solutions = {}  # final GPU iterates whose residual the CPU oracle re-computes
    if "mg" in sections:
        extra["mg_poisson_%d" % n] = mg_solves(P, torch, n, solutions)
    if "poisson" in sections and args.poisson_n > 0:
        names = {"jacobi": 0, "gs": 1, "rbgs": 2}
        methods = tuple(names[x] for x in args.poisson_methods.split(","))
        extra["poisson_%d" % args.poisson_n] = poisson_compare(
            P, torch, args.poisson_n, methods=methods, m=args.poisson_m,
            inners=tuple(args.poisson_inner.split(",")), keep=solutions)

    if "poisson" in sections:
        # the sizes the CPU oracle solves too (cpu_oracle_poisson_small)
        for ns in (32, 64):
            extra["poisson_%d" % ns] = poisson_compare(P, torch, ns, m=args.poisson_m)
    serving_sample = None
    if "serving" in sections and args.serving_jobs > 0:
        rates = [float(x) for x in str(args.serving_rate).split(",")]
        keep = tuple(range(0, args.serving_jobs, max(1, args.serving_jobs // 16)))[:16]
        runs, sjobs, sinputs, kept = serving_streams(P, args.serving_jobs, rates, keep=keep)
        extra["serving"] = runs[0] if len(runs) == 1 else runs
        serving_sample = (sjobs, sinputs, kept)

    line = {
        "metric": "MLUP/s & HBM-roofline fraction at 512^3 (FP64 vs FP32-refined); job p50/p99",
        "value": round(value, 1),
        "unit": "MLUP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "jacobi3d7pt_fp64_%d^3_x%d_sweeps" % (n, S), "interior": n,
                   "sweeps": S, "t_fuse": args.t, "plan": plan, "final_copy": fcopy,
                   "parallelism": "single-gpu"},
        "roofline": roof,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n)
        line["cpu_baseline"]["host"] = cpu_model()
        line["cpu_baseline"]["host_threads_available"] = os.cpu_count()
        extra["cpu_threads_baseline"] = cpu_threads_baseline(n)
        log("cpu threads baseline: %s" % extra["cpu_threads_baseline"])
        if "gs" in sections:
            extra["cpu_oracle_gs_384_x50"] = cpu_gs_oracle()
            log("cpu oracle gs: %s" % extra["cpu_oracle_gs_384_x50"])
        if "poisson" in sections:
            extra["cpu_oracle_poisson_small"] = cpu_refine_oracle()
        if solutions:
            extra["cpu_oracle_residual_of_gpu_solutions"] = cpu_residual_check(solutions)
            log("cpu oracle residuals: %s" % extra["cpu_oracle_residual_of_gpu_solutions"])
        if serving_sample is not None:
            sjobs, sinputs, kept = serving_sample
            extra["cpu_oracle_serving_sample"] = cpu_check_serving(sjobs, sinputs, kept)
            log("cpu oracle serving sample: %s" % extra["cpu_oracle_serving_sample"])
        extra["cpu_wavefront"] = cpu_wavefront(n)
        log("cpu wavefront: %s" % extra["cpu_wavefront"])
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
