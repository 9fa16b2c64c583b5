"""GPU parity for the FP64 residual, the refinement loop (FP32 inner smoother
inside FP64 defect correction, and the plain FP64 method) and the
continuous-batching job service."""
import math

import numpy as np
import pytest

import oracle
import synthetic_inputs as si
from gpu_util import assert_same, say, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def olib():
    oracle.build(force=False)
    return oracle.load()


@pytest.fixture(scope="module")
def P():
    torch_cuda()
    import paper_1004_1741_amd as P
    P.lib()
    return P


def _poisson(n_xyz, seed):
    nx, ny, nz = n_xyz
    f = si.uniform_rhs(nx, ny, nz, seed=seed)
    fp = f / float((max(n_xyz) + 1) ** 2)
    u = np.zeros(si.padded_shape(nx, ny, nz, 1))
    return u, fp


# --- residual -----------------------------------------------------------------

@pytest.mark.parametrize("dims", [(1, 1, 1), (7, 5, 3), (40, 33, 21), (130, 20, 9)])
def test_residual_parity(P, olib, dims):
    nx, ny, nz = dims
    u = si.uniform_padded(nx, ny, nz, 1, seed=nx, lo=-1.0, hi=1.0)
    fp = si.uniform_rhs(nx, ny, nz, seed=2)
    ref_r, ref_rr = oracle.residual(u, fp, lib=olib)
    import torch
    r = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    rr = P.residual(to_dev(u), to_dev(fp), r=r)
    assert_same(to_host(r), ref_r, "residual %s" % (dims,))
    assert abs(rr - ref_rr) <= 1e-12 * ref_rr


# --- refinement ---------------------------------------------------------------

@pytest.mark.parametrize("method", [0, 1, 2])
def test_refine_fp32_inner_fixed_steps(P, olib, method):
    """Three defect-correction steps, bit-exact against the oracle's loop."""
    u0, fp = _poisson((20, 17, 13), seed=3)
    u0[1:-1, 1:-1, 1:-1] = si.uniform_padded(20, 17, 13, 1, seed=4)[1:-1, 1:-1, 1:-1] * 1e-3
    ref, rc, outer, rel = oracle.refine(u0, fp, method=method, inner_f32=True, m=12, tol=0.0,
                                        max_outer=3, lib=olib)
    du = to_dev(u0)
    od, grel, grc = P.refine_solve(du, to_dev(fp), method=method, inner_fp32=True,
                                   inner_sweeps=12, rel_tol=0.0, max_outer=3,
                                   raise_on_noconv=False)
    assert grc == -6 and od == 3 and rc == -6 and outer == 3
    assert_same(to_host(du), ref, "refine fp32 inner method=%d" % method)
    assert abs(grel - rel) <= 1e-12 * rel


@pytest.mark.parametrize("method,m", [(0, 13), (2, 9)])
def test_refine_fp32_inner_odd_pass_count(P, olib, method, m):
    """Inner solves whose fused schedule has an odd number of passes (Jacobi
    13 = 6 + 6 + 1, red-black 9 = 3 + 3 + 3 at the FP32 defaults): the FP32
    correction and its scratch grid swap roles instead of a pass being split,
    and the swap carries into the next rounds.  Bit-exact against the
    oracle's loop."""
    u0, fp = _poisson((70, 61, 30), seed=12)
    ref, rc, outer, rel = oracle.refine(u0, fp, method=method, inner_f32=True, m=m, tol=0.0,
                                        max_outer=3, lib=olib)
    du = to_dev(u0)
    od, grel, grc = P.refine_solve(du, to_dev(fp), method=method, inner_fp32=True,
                                   inner_sweeps=m, rel_tol=0.0, max_outer=3,
                                   raise_on_noconv=False)
    assert grc == -6 and od == 3 and rc == -6 and outer == 3
    assert_same(to_host(du), ref, "refine fp32 odd passes method=%d m=%d" % (method, m))


@pytest.mark.parametrize("method", [0, 1, 2])
def test_refine_fp32_inner_fixed_steps_192(P, olib, method):
    """Two defect-correction steps on 192^3 (the float inner passes run
    interior tiles of the fused pass and the full wavefront), bit-exact
    against the oracle's loop."""
    n = 192
    u0, fp = _poisson((n, n, n), seed=8)
    m = 16
    assert P.jacobi_tiles(u0.shape, 6, fp32=True, rhs=True)[3] >= 1
    say("refine 192^3 fp32 inner method=%d (oracle)" % method)
    ref, rc, outer, rel = oracle.refine(u0, fp, method=method, inner_f32=True, m=m, tol=0.0,
                                        max_outer=2, lib=olib)
    du = to_dev(u0)
    say("refine 192^3 fp32 inner method=%d (GPU)" % method)
    od, grel, grc = P.refine_solve(du, to_dev(fp), method=method, inner_fp32=True,
                                   inner_sweeps=m, rel_tol=0.0, max_outer=2,
                                   raise_on_noconv=False)
    assert grc == -6 and od == 2 and rc == -6 and outer == 2
    assert_same(to_host(du), ref, "refine 192^3 fp32 inner method=%d" % method)
    assert abs(grel - rel) <= 1e-12 * rel


@pytest.mark.parametrize("method", [0, 1, 2])
def test_refine_plain_fp64_fixed_steps(P, olib, method):
    """The plain FP64 method: m sweeps of the smoother with f' between checks."""
    u0, fp = _poisson((18, 11, 16), seed=5)
    ref = u0.copy()
    for _ in range(3):
        ref = oracle.smooth(method, ref, 10, a=0.0, b=1.0 / 6.0, f=fp, g=1.0 / 6.0, lib=olib)
    du = to_dev(u0)
    od, _, grc = P.refine_solve(du, to_dev(fp), method=method, inner_fp32=False,
                                inner_sweeps=10, rel_tol=0.0, max_outer=3, raise_on_noconv=False)
    assert grc == -6 and od == 3
    assert_same(to_host(du), ref, "plain fp64 method=%d" % method)


@pytest.mark.parametrize("method", [0, 1, 2])
def test_refine_converges(P, olib, method):
    """FP32-refined solve reaches 1e-10; the oracle's residual of the GPU
    solution confirms it; the solution matches the plain FP64 solution."""
    n = 24
    u0, fp = _poisson((n, n, n), seed=6)
    du = to_dev(u0)
    say("refine converge method=%d" % method)
    od, rel, rc = P.refine_solve(du, to_dev(fp), method=method, inner_fp32=True,
                                 inner_sweeps=16, rel_tol=1e-10, max_outer=100000)
    assert rc == 0 and rel <= 1e-10
    got = to_host(du)
    _, rr = oracle.residual(got, fp, lib=olib)
    rel_cpu = math.sqrt(rr) / math.sqrt(oracle.sumsq(fp, lib=olib))
    assert rel_cpu <= 1e-10 * (1 + 1e-9), rel_cpu
    plain, prc, _, _ = oracle.refine(u0, fp, method=method, inner_f32=False, m=16, tol=1e-10,
                                     max_outer=100000, lib=olib)
    assert prc == 0
    # both satisfy ||r|| <= 1e-10 ||f'||; cond(A) < 12/(6-6cos(pi/25)) ~ 127
    scale = np.abs(plain).max()
    assert np.abs(got - plain).max() <= 2 * 127 * 1e-10 * scale * 10


def test_refine_noconv_reports(P):
    u0, fp = _poisson((10, 10, 10), seed=7)
    od, rel, rc = P.refine_solve(to_dev(u0), to_dev(fp), method=0, inner_fp32=True,
                                 inner_sweeps=4, rel_tol=1e-30, max_outer=2,
                                 raise_on_noconv=False)
    assert rc == -6 and od == 2 and 0 < rel < 1


# --- job service ----------------------------------------------------------------

def _jobs(seed=0, n=20):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nx, ny, nz = (int(v) for v in rng.integers(1, 41, size=3))
        method = int(rng.integers(0, 2))
        prec = int(rng.integers(0, 2))
        sweeps = int(rng.integers(0, 10))
        a, b = ((0.0, 1.0 / 6.0) if rng.random() < 0.7 else (0.2, 0.1))
        u = si.uniform_padded(nx, ny, nz, 1, seed=1000 + i)
        out.append(dict(u=u, method=method, prec=prec, sweeps=sweeps, a=a, b=b))
    return out


def _expected(j, olib):
    if j["prec"] == 0:
        return oracle.smooth(j["method"], j["u"], j["sweeps"], a=j["a"], b=j["b"], lib=olib)
    if j["sweeps"] == 0:
        return j["u"].copy()
    return oracle.refined_job(j["method"], j["u"], j["sweeps"], a=j["a"], b=j["b"], lib=olib)


def _serve(P, jobs, budget, max_inflight, sweeps_per_iteration=0):
    outs = [np.zeros_like(j["u"]) for j in jobs]
    with P.SmoothService(budget, max_inflight=max_inflight,
                         sweeps_per_iteration=sweeps_per_iteration) as svc:
        ids = [svc.submit(j["u"], o, j["sweeps"], method=j["method"], precision=j["prec"],
                          a=j["a"], b=j["b"]) for j, o in zip(jobs, outs)]
        svc.wait_all(timeout_ms=120000)
        states = [svc.poll(i) for i in ids]
        info = svc.info()
    return outs, states, info


def test_service_mixed_stream(P, olib):
    jobs = _jobs(seed=1, n=24)
    budget = 6 << 20  # forces queueing: several jobs wait for memory
    say("service: %d jobs, budget %d" % (len(jobs), budget))
    outs, states, info = _serve(P, jobs, budget, max_inflight=5)
    for k, (j, o, (st, stats)) in enumerate(zip(jobs, outs, states)):
        assert st == P.SmoothService.DONE, (k, st)
        exp = _expected(j, olib)
        assert_same(o, exp, "job %d (method %d prec %d sweeps %d)" % (k, j["method"], j["prec"],
                                                                    j["sweeps"]))
        if j["prec"] == 1 and j["sweeps"] > 0:
            plain = oracle.smooth(j["method"], j["u"], j["sweeps"], a=j["a"], b=j["b"], lib=olib)
            assert np.abs(o - plain).max() <= 1e-5 * max(1.0, np.abs(plain).max())
        assert stats.t_submit_ns <= stats.t_admit_ns <= stats.t_start_ns <= stats.t_done_ns
        assert stats.footprint_bytes > 0
    assert info.footprint_high_water <= budget
    assert info.max_resident_seen <= 5
    assert info.jobs_done == len(jobs) and info.jobs_failed == 0
    assert info.batches >= 1


@pytest.mark.parametrize("spi", [0, 3])
def test_service_alone_equals_mixed(P, olib, spi):
    """Each job gives the same result alone and in a mix, whether it runs all
    its sweeps in one iteration (0) or at most 3 per iteration; the mix also
    equals the oracle."""
    jobs = _jobs(seed=2, n=10)
    say("service alone vs mixed, sweeps_per_iteration=%d" % spi)
    mixed, states, info = _serve(P, jobs, 64 << 20, max_inflight=10, sweeps_per_iteration=spi)
    assert info.max_resident_seen >= 2  # jobs really shared iterations
    for k, j in enumerate(jobs):
        assert states[k][0] == P.SmoothService.DONE, k
        assert_same(mixed[k], _expected(j, olib), "job %d mixed vs oracle" % k)
        alone, st, _ = _serve(P, [j], 64 << 20, max_inflight=1, sweeps_per_iteration=spi)
        assert st[0][0] == P.SmoothService.DONE
        assert_same(alone[0], mixed[k], "job %d alone vs mixed" % k)


def test_service_errors(P):
    import paper_1004_1741_amd as PP
    svc = PP.SmoothService(1 << 20, max_inflight=2)
    try:
        big = np.zeros((130, 130, 130))
        with pytest.raises(PP.StencilError) as ei:
            svc.submit(big, np.zeros_like(big), 2)
        assert ei.value.status == PP.ST.EINVAL
        with pytest.raises(PP.StencilError) as ei:
            svc.poll(12345)
        assert ei.value.status == PP.ST.ENOENT
    finally:
        svc.shutdown()


def test_service_shutdown_cancels_pending(P, olib):
    """Queued jobs are cancelled (never written), resident ones drain to DONE."""
    first = si.uniform_padded(120, 120, 120, 1, seed=77)  # keeps the single slot busy
    small = [si.uniform_padded(16, 12, 10, 1, seed=78 + i) for i in range(8)]
    outs = [np.zeros_like(first)] + [np.zeros_like(u) for u in small]
    svc = P.SmoothService(64 << 20, max_inflight=1)
    svc.submit(first, outs[0], 50, method=0)
    for u, o in zip(small, outs[1:]):
        svc.submit(u, o, 3, method=1)
    svc.shutdown()
    assert_same(outs[0], oracle.jacobi(first, 50, lib=olib), "resident job drained")
    cancelled = 0
    for u, o in zip(small, outs[1:]):
        if not o.any():
            cancelled += 1  # never ran: output untouched
        else:
            assert_same(o, oracle.gauss_seidel(u, 3, lib=olib), "job done before shutdown")
    assert cancelled >= 1


def test_service_large_jobs_alone_mixed_oracle(P, olib):
    """Jobs of 130^3 and more (their passes run interior tiles of the batched
    kernels) next to small ones: each result is the same alone and in the mix,
    FP64 jobs equal the oracle bit for bit, FP32-refined jobs equal the
    oracle's emulation of the same steps and the plain result within 1e-5."""
    specs = [((140, 136, 132), 0, 0, 9), ((131, 150, 133), 1, 1, 7),
             ((133, 131, 140), 0, 1, 8), ((136, 140, 131), 1, 0, 5)]
    jobs = []
    for k, (dims, method, prec, sweeps) in enumerate(specs):
        jobs.append(dict(u=si.uniform_padded(*dims, 1, seed=500 + k), method=method, prec=prec,
                         sweeps=sweeps, a=0.0, b=1.0 / 6.0))
    jobs += _jobs(seed=9, n=6)
    say("service: %d jobs incl. four of >= 130^3" % len(jobs))
    mixed, states, info = _serve(P, jobs, 1 << 30, max_inflight=10)
    assert info.max_resident_seen >= 2
    for k, j in enumerate(jobs):
        assert states[k][0] == P.SmoothService.DONE, k
        assert_same(mixed[k], _expected(j, olib), "large-mix job %d vs oracle" % k)
        if j["prec"] == 1 and j["sweeps"] > 0:
            plain = oracle.smooth(j["method"], j["u"], j["sweeps"], a=j["a"], b=j["b"], lib=olib)
            assert np.abs(mixed[k] - plain).max() <= 1e-5 * max(1.0, np.abs(plain).max())
    for k in range(len(specs)):
        alone, st, _ = _serve(P, [jobs[k]], 1 << 30, max_inflight=1)
        assert st[0][0] == P.SmoothService.DONE
        assert_same(alone[0], mixed[k], "large job %d alone vs mixed" % k)
