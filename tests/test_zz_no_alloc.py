"""The allocation-free Gauss-Seidel entry point (stencil_gs_noalloc) against
stencil_gs: two calls in a row through the C ABI, the second on a smaller
grid, each bit-identical to stencil_gs on the same input.  The first call is
large enough that the workspace cap of the static device array splits its
sweeps over several launches; the second uses FP32 with a centre term and a
right-hand side.  Both are also checked against the oracle where it is quick."""
import numpy as np
import pytest

import oracle
import synthetic_inputs as si
from gpu_util import assert_same, say, to_dev, to_host, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    torch_cuda()
    import paper_1004_1741_amd as P
    P.lib()
    return P


def _both(P, u, sweeps, **kw):
    ref = to_dev(u)
    P.gauss_seidel(ref, sweeps, **kw)
    P.sync()
    got = to_dev(u)
    P.gauss_seidel_noalloc(got, sweeps, **kw)
    P.sync()
    return to_host(got), to_host(ref)


def test_gs_noalloc_two_calls(P):
    # call 1: 2048 x 2048 cross-section = 65536 bundles of 8x8 lines, so one
    # launch of the 4 MiB array holds at most 7 sweeps: 20 sweeps take 3 launches
    u1 = si.uniform_padded(24, 2048, 2048, 1, seed=11, lo=-1.0, hi=1.0)
    say("gs_noalloc call 1: 24x2048x2048 fp64 x20")
    got, ref = _both(P, u1, 20)
    assert_same(got, ref, "noalloc vs stencil_gs, 24x2048x2048 x20")
    del u1, got, ref
    # call 2: smaller, float, centre term and right-hand side, 3 sweeps per launch
    nx, ny, nz = 70, 50, 40
    u2 = si.uniform_padded(nx, ny, nz, 1, seed=12, lo=-1.0, hi=1.0).astype(np.float32)
    f2 = si.uniform_rhs(nx, ny, nz, seed=13).astype(np.float32)
    say("gs_noalloc call 2: 70x50x40 fp32 x7 with a and f")
    kw = dict(a=0.3, b=0.1, g=0.25, t_fuse=3)
    ref = to_dev(u2)
    P.gauss_seidel(ref, 7, f=to_dev(f2), **kw)
    P.sync()
    got = to_dev(u2)
    P.gauss_seidel_noalloc(got, 7, f=to_dev(f2), **kw)
    P.sync()
    assert_same(to_host(got), to_host(ref), "noalloc vs stencil_gs, 70x50x40 fp32 x7")
    assert_same(to_host(got), oracle.gauss_seidel(u2, 7, f=f2, a=0.3, b=0.1, g=0.25),
                "noalloc vs oracle, 70x50x40 fp32 x7")


def test_gs_noalloc_matches_oracle_fp64(P):
    u = si.gs_384(seed=5, n=96)["u"]
    say("gs_noalloc 96^3 fp64 x9 vs oracle")
    got, ref = _both(P, u, 9)
    assert_same(got, ref, "noalloc vs stencil_gs 96^3")
    assert_same(got, oracle.gauss_seidel(u, 9), "noalloc vs oracle 96^3")
