"""GPU parity: fused Jacobi passes and the Gauss-Seidel wavefront against the
CPU oracle, element by element, bit-exact (FP64 and FP32 alike: both sides
evaluate the Sec. 3 update in the same operand order without FMA)."""
import numpy as np
import pytest

import oracle
import synthetic_inputs as si
from gpu_util import assert_same, crop_for_sample, say, to_dev, to_host, torch_cuda

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


def _run_jacobi(P, u, sweeps, t, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1):
    du = to_dev(u)
    ds = to_dev(np.zeros_like(u))
    df = None if f is None else to_dev(f)
    P.jacobi(du, ds, sweeps, a=a, b=b, f=df, g=g, t_fuse=t, halo=h)
    return to_host(du)


def _run_gs(P, u, sweeps, t=0, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1):
    du = to_dev(u)
    df = None if f is None else to_dev(f)
    P.gauss_seidel(du, sweeps, a=a, b=b, f=df, g=g, t_fuse=t, halo=h)
    return to_host(du)


# --- the 64^3 workload: ghost 0, interior U[0,1), a=0, b=1/6, 10 sweeps -------

@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6, 7, 8, 16, 0])
def test_jacobi_64_all_t(P, olib, t):
    w = si.jacobi_small(seed=0)
    say("jacobi 64^3 x10 t=%d" % t)
    ref = oracle.jacobi(w["u"], w["sweeps"], a=w["a"], b=w["b"], lib=olib)
    got = _run_jacobi(P, w["u"], w["sweeps"], t)
    assert_same(got, ref, "jacobi 64^3 t=%d" % t)


# --- ragged and degenerate shapes, both dtypes, weights, RHS, wide ghosts -----

JAC_CASES = [
    # (nx, ny, nz, h, sweeps)
    (1, 1, 1, 1, 3),
    (2, 3, 5, 1, 4),
    (17, 63, 65, 1, 5),
    (130, 33, 7, 1, 9),
    (257, 5, 9, 2, 6),
    (119, 24, 40, 1, 8),    # x: two FP64 t=4 tiles of 56 and a ragged 7
    (245, 50, 19, 1, 13),
    (300, 70, 33, 1, 17),   # several tiles in x and y, several z-chunks
    (70, 61, 30, 3, 11),    # three ghost layers, boundary tiles on all sides,
                            # chunks long enough for steady-state steps
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", JAC_CASES, ids=lambda c: "x".join(map(str, c)))
def test_jacobi_ragged(P, olib, case, dtype):
    nx, ny, nz, h, S = case
    dt = np.float64 if dtype == "f64" else np.float32
    u = si.uniform_padded(nx, ny, nz, h, seed=nx + 7 * ny, lo=-1.0, hi=1.0).astype(dt)
    f = si.uniform_rhs(nx, ny, nz, seed=3).astype(dt)
    for t in range(1, 9):
        for (a, b, g, ff) in ((0.0, 1.0 / 6.0, 0.0, None), (0.3, 0.1, 0.25, f),
                              (0.0, 1.0 / 6.0, 1.0 / 6.0, f)):
            say("jacobi", case, dtype, "t=%d a=%g rhs=%s" % (t, a, ff is not None))
            ref = oracle.jacobi(u, S, a=a, b=b, f=ff, g=g, h=h, lib=olib)
            got = _run_jacobi(P, u, S, t, a=a, b=b, f=ff, g=g, h=h)
            assert_same(got, ref, "jacobi %s %s t=%d a=%g" % (case, dtype, t, a))


def test_jacobi_zero_sweeps_and_bc(P, olib):
    import paper_1004_1741_amd as PP
    u = si.uniform_padded(20, 10, 6, 1, seed=5)
    du, ds = to_dev(u), to_dev(np.zeros_like(u))
    PP.jacobi(du, ds, 0, bc=PP.ST.BC_CONST, bc_value=0.25)
    exp = si.set_ghosts(u.copy(), 1, 0.25)
    assert_same(to_host(du), exp, "bc fill only")
    PP.jacobi(du, ds, 3, bc=PP.ST.BC_CONST, bc_value=0.25)
    assert_same(to_host(du), oracle.jacobi(exp, 3, lib=olib), "bc fill + 3 sweeps")


@pytest.mark.parametrize("h", [2, 3])
def test_ghost_fill_and_copy_wide_halo(P, olib, h):
    """Ghost fill (BC_CONST) and the ghost copy into scratch with a halo wider
    than one: whole ghost rows and the 2h x ghosts of interior rows."""
    import paper_1004_1741_amd as PP
    u = si.uniform_padded(37, 11, 6, h, seed=21)
    du, ds = to_dev(u), to_dev(np.zeros_like(u))
    PP.jacobi(du, ds, 0, bc=PP.ST.BC_CONST, bc_value=-0.5, halo=h)
    exp = si.set_ghosts(u.copy(), h, -0.5)
    assert_same(to_host(du), exp, "bc fill only, h=%d" % h)
    PP.jacobi(du, ds, 5, t_fuse=1, halo=h)   # five one-sweep passes (odd count)
    assert_same(to_host(du), oracle.jacobi(exp, 5, h=h, lib=olib), "5 sweeps, h=%d" % h)


def test_jacobi_split_invariance(P, olib):
    u = si.uniform_padded(90, 40, 30, 1, seed=9)
    a = _run_jacobi(P, _run_jacobi(P, u, 7, 4), 6, 2)
    b = _run_jacobi(P, u, 13, 8)
    assert_same(a, b, "7+6 vs 13 sweeps")


# --- red-black Gauss-Seidel on the fused pass ----------------------------------

def _run_rbgs(P, u, sweeps, t, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1):
    du = to_dev(u)
    ds = to_dev(np.zeros_like(u))
    df = None if f is None else to_dev(f)
    P.red_black(du, ds, sweeps, a=a, b=b, f=df, g=g, t_fuse=t, halo=h)
    return to_host(du)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", JAC_CASES, ids=lambda c: "x".join(map(str, c)))
def test_rbgs_ragged(P, olib, case, dtype):
    nx, ny, nz, h, S = case
    dt = np.float64 if dtype == "f64" else np.float32
    u = si.uniform_padded(nx, ny, nz, h, seed=nx + 5 * nz, lo=-1.0, hi=1.0).astype(dt)
    f = si.uniform_rhs(nx, ny, nz, seed=4).astype(dt)
    for t in range(0, 5):
        for (a, b, g, ff) in ((0.0, 1.0 / 6.0, 0.0, None), (0.3, 0.1, 0.25, f),
                              (0.0, 1.0 / 6.0, 1.0 / 6.0, f)):
            say("red-black", case, dtype, "t=%d a=%g rhs=%s" % (t, a, ff is not None))
            ref = oracle.red_black(u, S, a=a, b=b, f=ff, g=g, h=h, lib=olib)
            got = _run_rbgs(P, u, S, t, a=a, b=b, f=ff, g=g, h=h)
            assert_same(got, ref, "red-black %s %s t=%d a=%g" % (case, dtype, t, a))


def test_rbgs_several_tiles_and_chunks(P, olib):
    """160 x 150 x 140 (ragged in every direction, several tiles and z-chunks),
    20 sweeps at the automatic depth and at 4 sweeps per pass."""
    u = si.uniform_padded(160, 150, 140, 1, seed=11)
    ref = oracle.red_black(u, 20, lib=olib)
    for t in (0, 4):
        say("red-black 160x150x140 x20 t=%d" % t)
        assert_same(_run_rbgs(P, u, 20, t), ref, "red-black 160x150x140 t=%d" % t)


@pytest.mark.parametrize("t", [0, 4])
def test_rbgs_512_sampled(P, olib, t):
    """The 512^3 grid of the benchmark, its tiling and z-chunks, 10 red-black
    sweeps, checked on 5^3 blocks of crops the oracle can afford.  A red-black
    sweep moves information two sites (red from black, black from the new
    red), so sites more than 2S from a cut face are exact; the crop origin
    keeps the colouring (crop and grid interior coordinates differ by an even
    sum)."""
    w = si.jacobi_512(seed=0)
    u = w["u"]
    S = 10
    say("red-black 512^3 x%d t=%d (GPU)" % (S, t))
    got = _run_rbgs(P, u, S, t)
    n = u.shape[0]
    m = 2 * S + 4  # block half-width 2, plus 2S + 2 to the cut faces
    for c in [(1, 1, 1), (1, n - 2, n // 2), (n // 2, n // 2, n // 2), (n - 2, 200, n - 2),
              (300, 1, 17), (77, 301, 455)]:
        lo = [max(0, x - m) for x in c]
        if sum(lo) % 2:  # keep the colouring: move one origin by one site
            ax = next(a for a in range(3) if lo[a] > 0) if any(lo) else 0
            lo[ax] -= 1
        sl = tuple(slice(lo[a], min(n, c[a] + m + 1)) for a in range(3))
        sub = np.ascontiguousarray(u[sl])
        blk = tuple(slice(max(0, c[a] - lo[a] - 2), c[a] - lo[a] + 3) for a in range(3))
        ref = oracle.red_black(sub, S, lib=olib)
        assert_same(got[sl][blk], ref[blk], "red-black 512^3 sample %s t=%d" % (c, t))
    assert np.isfinite(got).all()


def test_rbgs_differs_from_lexicographic(P, olib):
    u = si.uniform_padded(30, 20, 10, 1, seed=2)
    got = _run_rbgs(P, u, 3, 0)
    assert not np.array_equal(got, oracle.gauss_seidel(u, 3, lib=olib))


# --- full size: 512^3, 100 sweeps, sampled against the oracle -----------------

@pytest.mark.parametrize("t", [4, 5, 8])
def test_jacobi_512_sampled(P, olib, t):
    w = si.jacobi_512(seed=0)
    u = w["u"]
    S = w["sweeps"]
    say("jacobi 512^3 x100 t=%d (GPU)" % t)
    got = _run_jacobi(P, u, S, t)
    n = u.shape[0]
    # corner, edge, face and centre samples; each checked on its exact region
    centers = [(1, 1, 1), (1, n - 2, n // 2), (n // 2, n // 2, n // 2), (n - 2, 200, n - 2),
               (300, 1, 17)]
    for c in centers:
        sub, sl, inner = crop_for_sample(u, c, S)
        say("  oracle crop at", c, sub.shape)
        ref = oracle.jacobi(sub, S, lib=olib)
        g = got[sl]
        assert_same(g[inner], ref[inner], "512^3 sample %s" % (c,))
    # the whole result must still be finite and inside the data range
    assert np.isfinite(got).all()
    assert got.min() >= 0.0 and got.max() < 1.0


@pytest.mark.parametrize("t", [4, 5])
def test_jacobi_512_full_two_passes(P, olib, t):
    """The whole 512^3 grid after two passes of depth t, element by element:
    every tile overlap and z-chunk seam of the benchmark's launch shape."""
    w = si.jacobi_512(seed=0)
    u = w["u"]
    S = 2 * t
    say("jacobi 512^3 x%d t=%d, whole grid (GPU)" % (S, t))
    got = _run_jacobi(P, u, S, t)
    say("  oracle 512^3 x%d" % S)
    ref = oracle.jacobi(u, S, lib=olib)
    assert_same(got, ref, "512^3 x%d t=%d whole grid" % (S, t))


# --- Gauss-Seidel ---------------------------------------------------------------

GS_CASES = [
    (8, 8, 8, 1, 1),
    (8, 8, 8, 1, 3),
    (1, 1, 1, 1, 2),
    (5, 9, 17, 1, 3),
    (33, 20, 17, 1, 4),
    (64, 24, 40, 2, 3),
    (100, 30, 9, 1, 5),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", GS_CASES, ids=lambda c: "x".join(map(str, c)))
def test_gs_ragged(P, olib, case, dtype):
    nx, ny, nz, h, S = case
    dt = np.float64 if dtype == "f64" else np.float32
    u = si.uniform_padded(nx, ny, nz, h, seed=11 + nx, lo=-1.0, hi=1.0).astype(dt)
    f = si.uniform_rhs(nx, ny, nz, seed=4).astype(dt)
    for (a, b, g, ff) in ((0.0, 1.0 / 6.0, 0.0, None), (0.2, 0.125, 0.5, f)):
        for t in (0, 1):
            say("gs", case, dtype, "a=%g rhs=%s t=%d" % (a, ff is not None, t))
            ref = oracle.gauss_seidel(u, S, a=a, b=b, f=ff, g=g, h=h, lib=olib)
            got = _run_gs(P, u, S, t, a=a, b=b, f=ff, g=g, h=h)
            assert_same(got, ref, "gs %s %s a=%g t=%d" % (case, dtype, a, t))


def test_gs_96_many_sweeps(P, olib):
    u = si.gs_384(seed=1, n=96)["u"]
    say("gs 96^3 x12")
    ref = oracle.gauss_seidel(u, 12, lib=olib)
    for t in (0, 1, 4):
        assert_same(_run_gs(P, u, 12, t), ref, "gs 96^3 t=%d" % t)


def test_gs_384_full(P, olib):
    w = si.gs_384(seed=0)
    say("gs 384^3 x50 (GPU)")
    got = _run_gs(P, w["u"], w["sweeps"], 0)
    say("gs 384^3 x50 (oracle)")
    ref = oracle.gauss_seidel(w["u"], w["sweeps"], lib=olib)
    assert_same(got, ref, "gs 384^3 x50")
