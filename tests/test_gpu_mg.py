"""Multigrid V-cycles on the GPU (stencil_mg_solve) against the oracle.

A fixed number of V-cycles (rel_tol = 0) must give the oracle's result bit
for bit: every smoother (weighted Jacobi through the fused pass, the
Gauss-Seidel wavefront, the red-black pass), FP32 and FP64 inner cycles,
nested (n+1 even) and non-nested (n+1 odd) level hierarchies, non-cubic and
ragged grids and a wide ghost layer.  Converged solves are checked by the
oracle's own residual of the GPU solution, at 127^3 and at the full 512^3
Poisson workload (f' = f/513^2, f U[-1,1) seed 0), where two V-cycles are
also compared element by element."""
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


def _problem(nx, ny, nz, h, seed):
    f = si.uniform_rhs(nx, ny, nz, seed=seed)
    fp = f / float((max(nx, ny, nz) + 1) ** 2)
    u = np.zeros((nz + 2 * h, ny + 2 * h, nx + 2 * h))
    return u, fp


CASES = [  # nx, ny, nz, halo
    (31, 31, 31, 1),     # nested to 1^3
    (33, 20, 17, 1),     # non-nested, non-cubic, ragged tiles
    (64, 48, 40, 1),     # several tiles per level
    (22, 18, 26, 2),     # wide ghost layer on the finest level
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
@pytest.mark.parametrize("smoother", [0, 1, 2])
@pytest.mark.parametrize("inner_fp32", [True, False], ids=["fp32", "fp64"])
def test_mg_fixed_cycles_bit_exact(P, olib, case, smoother, inner_fp32):
    nx, ny, nz, h = case
    u, fp = _problem(nx, ny, nz, h, seed=nx + 3 * smoother)
    cycles = 3
    say("mg %s smoother=%d fp32=%s x%d cycles" % (case, smoother, inner_fp32, cycles))
    ref, rc, cyc, rel, _ = oracle.mg_solve(u, fp, smoother=smoother, inner_f32=inner_fp32, pre=2,
                                           post=1, coarse=9, tol=0.0, max_cycles=cycles, h=h,
                                           lib=olib)
    assert cyc == cycles
    du = to_dev(u)
    got_cyc, got_rel, st = P.mg_solve(du, to_dev(fp), smoother=smoother, inner_fp32=inner_fp32,
                                      pre=2, post=1, coarse_sweeps=9, rel_tol=0.0,
                                      max_cycles=cycles, halo=h, raise_on_noconv=False)
    assert st == P.ST.ENOCONV and got_cyc == cycles
    assert_same(to_host(du), ref, "mg %s sm=%d fp32=%s" % (case, smoother, inner_fp32))
    assert abs(got_rel - rel) <= 1e-12 * rel


@pytest.mark.parametrize("smoother", [0, 1, 2])
def test_mg_converges_127(P, olib, smoother):
    n = 127
    u, fp = _problem(n, n, n, 1, seed=9)
    du = to_dev(u)
    say("mg 127^3 smoother=%d to 1e-10" % smoother)
    cyc, rel, st = P.mg_solve(du, to_dev(fp), smoother=smoother, rel_tol=1e-10, max_cycles=40)
    assert st == 0 and rel <= 1e-10 and cyc <= 25, (cyc, rel)
    _, rr = oracle.residual(to_host(du), fp, lib=olib)
    assert np.sqrt(rr) / np.sqrt(oracle.sumsq(fp, lib=olib)) <= 1.0001e-10


def test_mg_poisson_512(P, olib):
    """The 512^3 Poisson workload: two red-black V(2,2) cycles in float are
    bit-identical to the oracle's; the converged FP32-inner solve has an
    oracle residual below 1e-10."""
    w = si.poisson(512, seed=0)
    fp = w["f"] / 513.0 ** 2
    dfp = to_dev(fp)
    du = to_dev(w["u"])
    say("mg 512^3 two cycles (GPU)")
    cyc, rel, st = P.mg_solve(du, dfp, smoother=2, rel_tol=0.0, max_cycles=2,
                              raise_on_noconv=False)
    assert cyc == 2
    got = to_host(du)
    say("  oracle")
    ref, _, _, orel, _ = oracle.mg_solve(w["u"], fp, smoother=2, inner_f32=True, pre=2, post=2,
                                         coarse=16, tol=0.0, max_cycles=2, lib=olib)
    assert_same(got, ref, "mg 512^3 x2 cycles")
    del got, ref
    say("mg 512^3 to 1e-10 (GPU)")
    du = to_dev(w["u"])
    cyc, rel, st = P.mg_solve(du, dfp, smoother=2, rel_tol=1e-10, max_cycles=40)
    assert st == 0 and rel <= 1e-10 and cyc <= 20, (cyc, rel)
    _, rr = oracle.residual(to_host(du), fp, lib=olib)
    orel = np.sqrt(rr) / np.sqrt(oracle.sumsq(fp, lib=olib))
    say("  %d cycles, GPU rel %.3e, oracle rel %.3e" % (cyc, rel, orel))
    assert orel <= 1.0001e-10
