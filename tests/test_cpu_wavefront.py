"""The paper's multicore schemes on the host CPU (cpu_baseline/wavefront.c)
against the oracle, bit for bit: the Sec. 4 temporal wavefront Jacobi with
skewed y-blocks and boundary arrays, and the Sec. 3 pipeline-parallel
Gauss-Seidel combined with the Sec. 4 wavefront.  Only the order of
independent site updates differs from the plain loop nests, so every
configuration (depth, thread groups, block height, sub-blocks, ghost width,
centre term, right-hand side, remainder passes) must give identical bits."""
import numpy as np
import pytest

import cpu_baseline as W
import oracle

GRIDS = [(13, 37, 11, 1), (20, 17, 9, 2), (5, 5, 5, 1), (31, 64, 20, 1), (9, 3, 6, 1)]
WEIGHTS = [(0.0, 1.0 / 6.0, 0.0, False), (0.3, 0.1, 0.25, True)]


@pytest.fixture(scope="module", autouse=True)
def _built():
    W.build(force=False)


def _inputs(nx, ny, nz, h, seed):
    rng = np.random.default_rng(seed)
    u = rng.random((nz + 2 * h, ny + 2 * h, nx + 2 * h))
    f = 2.0 * rng.random((nz, ny, nx)) - 1.0
    return u, f


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: "x".join(map(str, g)))
@pytest.mark.parametrize("t", [1, 2, 3, 4, 6])
def test_wavefront_jacobi_matches_oracle(grid, t):
    nx, ny, nz, h = grid
    u, f = _inputs(nx, ny, nz, h, seed=nx * 7 + t)
    for sweeps in (1, t, 2 * t + 1):
        for groups, block_y in ((1, 1), (2, 6), (3, 10)):
            for a, b, g, use_f in WEIGHTS:
                ff = f if use_f else None
                ref = oracle.jacobi(u, sweeps, a=a, b=b, f=ff, g=g, h=h)
                got = W.jacobi(u, sweeps, t=t, groups=groups, block_y=block_y, a=a, b=b, f=ff,
                               g=g, h=h)
                assert np.array_equal(got, ref), (grid, t, sweeps, groups, block_y, a)


@pytest.mark.parametrize("grid", GRIDS, ids=lambda g: "x".join(map(str, g)))
@pytest.mark.parametrize("t,P", [(1, 1), (1, 4), (2, 3), (3, 2), (4, 5)])
def test_pipeline_gs_matches_oracle(grid, t, P):
    nx, ny, nz, h = grid
    u, f = _inputs(nx, ny, nz, h, seed=ny * 5 + P)
    for sweeps in (1, 2 * t + 1):
        for a, b, g, use_f in WEIGHTS:
            ff = f if use_f else None
            ref = oracle.gauss_seidel(u, sweeps, a=a, b=b, f=ff, g=g, h=h)
            got = W.gauss_seidel(u, sweeps, t=t, subblocks=P, a=a, b=b, f=ff, g=g, h=h)
            assert np.array_equal(got, ref), (grid, t, P, sweeps, a)


def test_wavefront_many_threads_medium_grid():
    """A grid with many y-blocks per group and more threads than this machine
    may have cores (the barrier yields): 4 groups of depth 4."""
    u, _ = _inputs(40, 96, 30, 1, seed=3)
    ref = oracle.jacobi(u, 9)
    assert np.array_equal(W.jacobi(u, 9, t=4, groups=4, block_y=8), ref)
    refg = oracle.gauss_seidel(u, 6)
    assert np.array_equal(W.gauss_seidel(u, 6, t=3, subblocks=6), refg)


def test_zero_sweeps_and_bad_arguments():
    u, _ = _inputs(6, 6, 6, 1, seed=0)
    assert np.array_equal(W.jacobi(u, 0), u)
    assert np.array_equal(W.gauss_seidel(u, 0), u)
    with pytest.raises(ValueError):
        W.jacobi(u, 1, t=0)
    with pytest.raises(ValueError):
        W.gauss_seidel(u, 1, subblocks=0)
    assert W.cpu_count() >= 1
