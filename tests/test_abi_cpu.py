"""Host-side checks of the C ABI (no GPU work): exported symbols, argument
validation before anything is enqueued, the pass planner, the pool
allocator, and the Eq. (1) bandwidth model used by bench.py."""
import ctypes
import json
import pathlib
import re
import subprocess
import sys

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "stencil.h"


@pytest.fixture(scope="module")
def P():
    import paper_1004_1741_amd as P
    if not P.LIB_PATH.exists():
        from paper_1004_1741_amd import build
        build.build()
    P.lib()
    return P


def declared_functions():
    text = re.sub(r"/\*.*?\*/", "", HEADER.read_text(), flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("stencil_", "smooth_"))))


def test_header_symbols_exported(P):
    names = declared_functions()
    assert len(names) >= 14, names
    out = subprocess.run(["nm", "-D", "--defined-only", str(P.LIB_PATH)], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    bound = set(n for n, _, _ in P.SIGNATURES)
    assert set(names) == bound, set(names) ^ bound


def _grid(P, nx=8, ny=8, nz=8, h=1):
    return P.Grid(nx, ny, nz, h)


FAKE = ctypes.c_void_p(0x10000)   # never dereferenced: every call below fails validation
FAKE2 = ctypes.c_void_p(0x90000000)


@pytest.mark.parametrize("kw,status", [
    (dict(nx=0), -1), (dict(h=0), -1), (dict(dtype=7), -1), (dict(u=None), -1),
    (dict(scratch=None), -1), (dict(t=9), -1), (dict(sweeps=-1), -1), (dict(bc=9), -1),
    (dict(overlap=True), -1), (dict(w=None), -1), (dict(nx=1 << 40), -1),
])
def test_jacobi_validation(P, kw, status):
    L = P.lib()
    g = _grid(P, nx=kw.get("nx", 8), h=kw.get("h", 1))
    w = None if "w" in kw else ctypes.byref(P.Weights(0.0, 1.0 / 6.0, 0.0))
    u = kw.get("u", FAKE)
    s = FAKE if kw.get("overlap") else kw.get("scratch", FAKE2)
    rc = L.stencil_jacobi(ctypes.byref(g), kw.get("dtype", 0), u, s, None, w, kw.get("bc", 0), 0.0,
                          kw.get("sweeps", 1), kw.get("t", 0), None)
    assert rc == status
    assert L.stencil_last_error()


@pytest.mark.parametrize("nx,ny", [(16382, 16382), ((1 << 26) - 2, 2), (2, (1 << 27) - 2)])
def test_plane_size_limit(P, nx, ny):
    """A padded plane of 2^28 or more elements is rejected before any device
    call (kernels address a plane with 32-bit byte offsets)."""
    L = P.lib()
    g = P.Grid(nx, ny, 4, 1)
    w = ctypes.byref(P.Weights(0.0, 1.0 / 6.0, 0.0))
    for fn in (L.stencil_jacobi, L.stencil_rbgs):
        rc = fn(ctypes.byref(g), 0, FAKE, FAKE2, None, w, 0, 0.0, 1, 0, None)
        assert rc == P.ST.EINVAL
        assert b"2^28" in L.stencil_last_error()
    rc = L.stencil_gs(ctypes.byref(g), 0, FAKE, None, w, 0, 0.0, 1, 0, None)
    assert rc == P.ST.EINVAL


@pytest.mark.parametrize("kw,status", [
    (dict(nx=0), -1), (dict(dtype=7), -1), (dict(u=None), -1), (dict(scratch=None), -1),
    (dict(t=5), -1), (dict(t=-1), -1), (dict(sweeps=-1), -1), (dict(bc=9), -1),
    (dict(overlap=True), -1), (dict(w=None), -1),
])
def test_rbgs_validation(P, kw, status):
    L = P.lib()
    g = _grid(P, nx=kw.get("nx", 8))
    w = None if "w" in kw else ctypes.byref(P.Weights(0.0, 1.0 / 6.0, 0.0))
    u = kw.get("u", FAKE)
    s = FAKE if kw.get("overlap") else kw.get("scratch", FAKE2)
    rc = L.stencil_rbgs(ctypes.byref(g), kw.get("dtype", 0), u, s, None, w, kw.get("bc", 0), 0.0,
                        kw.get("sweeps", 1), kw.get("t", 0), None)
    assert rc == status
    assert L.stencil_last_error()


@pytest.mark.parametrize("kw", [dict(nz=0), dict(dtype=2), dict(u=None), dict(t=11),
                                dict(sweeps=-3), dict(ny=9000)])
def test_gs_validation(P, kw):
    L = P.lib()
    g = _grid(P, ny=kw.get("ny", 8), nz=kw.get("nz", 8))
    w = P.Weights(0.0, 1.0 / 6.0, 0.0)
    rc = L.stencil_gs(ctypes.byref(g), kw.get("dtype", 0), kw.get("u", FAKE), None, ctypes.byref(w),
                      0, 0.0, kw.get("sweeps", 1), kw.get("t", 0), None)
    assert rc == P.ST.EINVAL


@pytest.mark.parametrize("kw", [dict(nz=0), dict(dtype=2), dict(u=None), dict(t=11),
                                dict(sweeps=-3), dict(ny=9000), dict(ny=6000, nz=6000)])
def test_gs_noalloc_validation(P, kw):
    """The allocation-free entry point rejects what stencil_gs rejects, and a
    grid whose one-sweep workspace exceeds its static device array, before
    any device call."""
    L = P.lib()
    g = _grid(P, ny=kw.get("ny", 8), nz=kw.get("nz", 8))
    w = P.Weights(0.0, 1.0 / 6.0, 0.0)
    rc = L.stencil_gs_noalloc(ctypes.byref(g), kw.get("dtype", 0), kw.get("u", FAKE), None,
                              ctypes.byref(w), 0, 0.0, kw.get("sweeps", 1), kw.get("t", 0), None)
    assert rc == P.ST.EINVAL
    if kw.get("ny") == 6000:
        assert b"4 MiB" in L.stencil_last_error()


def test_refine_and_residual_validation(P):
    L = P.lib()
    g = _grid(P)
    od, rel = ctypes.c_int32(0), ctypes.c_double(0)
    args = dict(method=0, dt=1, u=FAKE, fp=FAKE2, m=4, t=0, tol=1e-10, mo=5)
    for bad in (dict(method=3), dict(method=2, t=5), dict(dt=3), dict(u=None), dict(fp=None),
                dict(m=0), dict(t=10),
                dict(tol=-1.0), dict(mo=-1)):
        a = dict(args, **bad)
        rc = L.stencil_refine_solve(ctypes.byref(g), a["method"], a["dt"], a["u"], a["fp"], a["m"],
                                    a["t"], a["tol"], a["mo"], ctypes.byref(od), ctypes.byref(rel),
                                    None)
        assert rc == P.ST.EINVAL, bad
    assert L.stencil_residual(ctypes.byref(g), FAKE, None, None, None, None) == P.ST.EINVAL
    assert L.stencil_residual(ctypes.byref(_grid(P, nx=0)), FAKE, None, None,
                              ctypes.byref(rel), None) == P.ST.EINVAL


def test_service_validation(P):
    L = P.lib()
    ctx = ctypes.c_void_p(None)
    assert L.smooth_init(ctypes.byref(P.SmoothConfig(1 << 20, 0, 0, 0, 0)),
                         ctypes.byref(ctx)) == P.ST.EINVAL
    assert L.smooth_init(ctypes.byref(P.SmoothConfig(1 << 20, 4, 0, 9, 0)),
                         ctypes.byref(ctx)) == P.ST.EINVAL
    assert L.smooth_init(ctypes.byref(P.SmoothConfig(1 << 20, 4, 0, 0, -1)),
                         ctypes.byref(ctx)) == P.ST.EINVAL
    assert L.smooth_init(None, ctypes.byref(ctx)) == P.ST.EINVAL
    jid = ctypes.c_uint64(0)
    st = ctypes.c_int32(0)
    assert L.smooth_submit(None, None, ctypes.byref(jid)) == P.ST.EINVAL
    assert L.smooth_poll(None, 1, ctypes.byref(st), None) == P.ST.EINVAL
    assert L.smooth_wait_all(None, 0) == P.ST.EINVAL
    assert L.smooth_shutdown(None) == P.ST.EINVAL


def test_strerror(P):
    L = P.lib()
    names = {0: b"ok", -1: b"invalid argument", -2: b"out of memory", -3: b"HIP runtime error",
             -4: b"busy", -5: b"no such job", -6: b"not converged", -7: b"canceled"}
    for code, name in names.items():
        assert L.stencil_strerror(code) == name
    assert L.stencil_strerror(99) == b"unknown status"


@pytest.mark.parametrize("fp32", [False, True])
def test_jacobi_plan(P, fp32):
    """Every schedule sums to the sweep count, uses only compiled depths, and
    leaves the result in u (even pass count) unless only 1-sweep passes exist."""
    auto = max(P.jacobi_plan(40, 0, fp32=fp32)[0])
    assert 1 <= auto <= 8
    assert P.jacobi_plan(100, 0, fp32=fp32)[0] == [5] * 20
    assert max(P.jacobi_plan(40, 0, fp32=fp32, rhs=True)[0]) == (6 if fp32 else 4)
    for S in list(range(0, 40)) + [64, 99, 100, 101, 255]:
        for t in (0, 1, 2, 3, 4, 5, 6, 7, 8, 16):
            plan, fc = P.jacobi_plan(S, t, fp32=fp32)
            assert sum(plan) == S
            tmax = {0: auto, 16: 8}.get(t, t)
            assert all(1 <= p <= tmax for p in plan)
            if fc:
                assert len(plan) % 2 == 1 and all(p == 1 for p in plan)
            else:
                assert len(plan) % 2 == 0
    plan, _ = P.jacobi_plan(100, 4)
    assert len(plan) == 26  # 25 passes of 4, odd: one of them split in two
    plan, _ = P.jacobi_plan(100, 5)
    assert plan == [5] * 20
    plan, fc = P.jacobi_plan(13, 5)
    assert sorted(plan) == [1, 2, 5, 5] and not fc  # 5+5+3, the 3 split as 2+1
    for bad in (-1, 9, 12, 17):
        with pytest.raises(Exception):
            P.jacobi_plan(10, bad)


def test_pool_allocator(tmp_path):
    exe = tmp_path / "pool_test"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", str(ROOT / "paper_1004_1741_amd" / "csrc"),
                    str(ROOT / "tests" / "native" / "pool_test.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "pool ok" in r.stdout


def test_eq1_model_against_table1():
    """Eq. (1) with Table 1's STREAM bandwidths; the paper's measured 1008
    MLUP/s (threaded Nehalem EP, non-temporal stores, Sec. 4) must sit below
    its Eq. (1) limit and close to it (memory-bound)."""
    sys.path.insert(0, str(ROOT))
    import bench
    d = json.loads((ROOT / "tests" / "golden" / "eq1_table1.json").read_text())
    for m in d["machines"]:
        lim = bench.eq1_mlups(m["stream_nt_GBs"])
        assert abs(lim * 16 - m["stream_nt_GBs"] * 1000) < 1e-6
        assert bench.eq1_mlups(m["stream_nt_GBs"], t=4) == pytest.approx(4 * lim)
        assert bench.eq1_mlups(m["stream_nt_GBs"], elem_bytes=4) == pytest.approx(2 * lim)
    ep = d["machines"][1]
    lim = bench.eq1_mlups(ep["stream_nt_GBs"])
    meas = d["measured_nehalem_ep_jacobi_threaded_mlups"]
    assert 0.8 * lim <= meas <= lim
    assert bench.bytes_per_lup(8, 1) == 16.0 and bench.bytes_per_lup(8, 8) == 2.0


def test_bench_refuses_multi_gpu():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
