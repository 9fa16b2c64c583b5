"""GPU parity that reaches every compiled variant of the fused pass.

A tile of the fused pass takes the unmasked (interior) code path only when its
whole loaded footprint lies inside the interior, and the masked (edge) path
otherwise; the two paths load, mask and store differently.  The tests below
run every dtype x level count x (centre term, right-hand side) instantiation
of the Jacobi pass and of the red-black pass on a grid where the library's
own tile count (stencil_jacobi_tiles) reports at least one tile of each kind,
and compare the whole result with the oracle, bit for bit.  Full-size checks
follow: the whole 512^3 grid in float after two passes (t = 5 without and
t = 6 with a right-hand side), FP64 with a right-hand side at t = 4, and the
Gauss-Seidel wavefront at 512^3.  The last tests cover the bounded waits of
the wavefront (forced from the host: a one-poll spin limit and the abort
word), after which the same launch is bit-exact again.
"""
import numpy as np
import pytest

import oracle
import synthetic_inputs as si
from gpu_util import assert_same, say, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu

# 252 x 254 x 13: every (dtype, levels, rhs) tiling has interior and edge tiles
COVER = (252, 254, 13)
WEIGHTS = [  # (a, b, g, use_f)
    (0.0, 1.0 / 6.0, 0.0, False),
    (0.3, 0.1, 0.25, True),
    (0.0, 1.0 / 6.0, 1.0 / 6.0, True),
    (0.25, 0.125, 0.0, False),
]


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


def _tiles_ok(P, shape, levels, fp32, rhs):
    tw, th, nt, ni = P.jacobi_tiles(shape, levels, fp32=fp32, rhs=rhs)
    assert ni >= 1 and nt - ni >= 1, ("grid does not reach both tile kinds", shape, levels,
                                      fp32, rhs, (tw, th, nt, ni))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6, 7, 8])
def test_jacobi_interior_and_edge_tiles(P, olib, dtype, t):
    nx, ny, nz = COVER
    dt = np.float64 if dtype == "f64" else np.float32
    u = si.uniform_padded(nx, ny, nz, 1, seed=31 + t, lo=-1.0, hi=1.0).astype(dt)
    f = si.uniform_rhs(nx, ny, nz, seed=32).astype(dt)
    S = 2 * t + 1  # two full passes and a remainder pass
    for a, b, g, use_f in WEIGHTS:
        _tiles_ok(P, u.shape, t, dtype == "f32", use_f)
        ff = f if use_f else None
        say("jacobi cover %s t=%d a=%g rhs=%s" % (dtype, t, a, use_f))
        ref = oracle.jacobi(u, S, a=a, b=b, f=ff, g=g, lib=olib)
        du, ds = to_dev(u), to_dev(np.zeros_like(u))
        P.jacobi(du, ds, S, a=a, b=b, f=None if ff is None else to_dev(ff), g=g, t_fuse=t)
        assert_same(to_host(du), ref, "jacobi cover %s t=%d a=%g rhs=%s" % (dtype, t, a, use_f))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("t", [1, 2, 3, 4])
def test_rbgs_interior_and_edge_tiles(P, olib, dtype, t):
    nx, ny, nz = COVER
    dt = np.float64 if dtype == "f64" else np.float32
    u = si.uniform_padded(nx, ny, nz, 1, seed=41 + t, lo=-1.0, hi=1.0).astype(dt)
    f = si.uniform_rhs(nx, ny, nz, seed=42).astype(dt)
    S = 2 * t + 1
    for a, b, g, use_f in WEIGHTS:
        _tiles_ok(P, u.shape, 2 * t, dtype == "f32", use_f)
        ff = f if use_f else None
        say("red-black cover %s t=%d a=%g rhs=%s" % (dtype, t, a, use_f))
        ref = oracle.red_black(u, S, a=a, b=b, f=ff, g=g, lib=olib)
        du, ds = to_dev(u), to_dev(np.zeros_like(u))
        P.red_black(du, ds, S, a=a, b=b, f=None if ff is None else to_dev(ff), g=g, t_fuse=t)
        assert_same(to_host(du), ref, "red-black cover %s t=%d a=%g rhs=%s" % (dtype, t, a, use_f))


# --- whole 512^3 grids -------------------------------------------------------

@pytest.mark.parametrize("case", [("f32", 5, False), ("f32", 6, True), ("f64", 4, True)],
                         ids=lambda c: "%s_t%d_%s" % (c[0], c[1], "rhs" if c[2] else "norhs"))
def test_jacobi_512_whole_grid(P, olib, case):
    """Two passes of depth t over the whole 512^3 grid (the launch shape of the
    benchmark and of the FP32 inner solve), compared element by element."""
    dtype, t, use_f = case
    dt = np.float64 if dtype == "f64" else np.float32
    u = si.jacobi_512(seed=0)["u"].astype(dt)
    f = si.uniform_rhs(512, 512, 512, seed=0).astype(dt) if use_f else None
    g = 1.0 / 6.0 if use_f else 0.0
    _tiles_ok(P, u.shape, t, dtype == "f32", use_f)
    S = 2 * t
    say("jacobi 512^3 %s x%d t=%d rhs=%s (GPU)" % (dtype, S, t, use_f))
    du, ds = to_dev(u), to_dev(np.zeros_like(u))
    P.jacobi(du, ds, S, f=None if f is None else to_dev(f), g=g, t_fuse=t)
    got = to_host(du)
    del du, ds
    say("  oracle")
    ref = oracle.jacobi(u, S, f=f, g=g, lib=olib)
    assert_same(got, ref, "512^3 %s x%d t=%d rhs=%s" % (dtype, S, t, use_f))


def test_gs_512_whole_grid(P, olib):
    """The Gauss-Seidel wavefront on 512^3 (FP64, four sweeps in flight),
    element by element against the sequential loop nest."""
    g = si.gs_384(seed=0, n=512)
    S = 4
    say("gs 512^3 x%d (GPU)" % S)
    du = to_dev(g["u"])
    P.gauss_seidel(du, S)
    P.sync()
    got = to_host(du)
    del du
    say("  oracle")
    ref = oracle.gauss_seidel(g["u"], S, lib=olib)
    assert_same(got, ref, "gs 512^3 x%d" % S)


# --- bounded waits of the wavefront -------------------------------------------

def test_gs_spin_limit_gives_up_and_recovers(P, olib):
    """A one-poll limit makes the first unsatisfied wait give up: the launch
    ends normally, sync() reports it, and the same launch is bit-exact after
    the default limit is restored."""
    import paper_1004_1741_amd as PP
    u = si.gs_384(seed=3, n=96)["u"]
    ref = oracle.gauss_seidel(u, 12, lib=olib)
    du = to_dev(u)
    PP.sync()
    PP.gs_spin_limit(1)
    try:
        say("gs 96^3 x12 with a one-poll spin limit")
        PP.gauss_seidel(du, 12)
        with pytest.raises(PP.StencilError) as ei:
            PP.sync()
        assert ei.value.status == PP.ST.EHIP
    finally:
        PP.gs_spin_limit(0)
    PP.sync()  # cleared
    du = to_dev(u)
    PP.gauss_seidel(du, 12)
    PP.sync()
    assert_same(to_host(du), ref, "gs 96^3 after recovery")


def test_gs_abort_word_from_host(P, olib):
    """The host raises the abort word: the next launch gives up at its first
    wait and exits; sync() reports it and clears the word."""
    import paper_1004_1741_amd as PP
    u = si.gs_384(seed=4, n=64)["u"]
    ref = oracle.gauss_seidel(u, 6, lib=olib)
    PP.sync()
    PP.gs_abort(0)
    du = to_dev(u)
    say("gs 64^3 x6 with the abort word raised")
    PP.gauss_seidel(du, 6)
    with pytest.raises(PP.StencilError) as ei:
        PP.sync()
    assert ei.value.status == PP.ST.EHIP
    du = to_dev(u)
    PP.gauss_seidel(du, 6)
    PP.sync()
    assert_same(to_host(du), ref, "gs 64^3 after abort cleared")
