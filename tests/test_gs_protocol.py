"""The Gauss-Seidel wavefront protocol, emulated on the CPU (no GPU)."""
import numpy as np
import pytest

import gs_protocol_model as M
import oracle
import synthetic_inputs as si


@pytest.mark.parametrize("dims,S,workers,seed", [
    ((9, 8, 8), 2, 2, 0), ((5, 9, 17), 3, 3, 1), ((1, 1, 1), 2, 2, 3), ((16, 16, 9), 4, 1, 4),
    ((24, 11, 19), 2, 7, 5), ((100, 30, 9), 5, 16, 2),
])
def test_protocol_matches_sequential_sweeps(dims, S, workers, seed):
    nx, ny, nz = dims
    u0 = si.uniform_padded(nx, ny, nz, 1, seed=seed, lo=-1.0, hi=1.0)
    got = M.simulate(u0, S, workers=workers, seed=seed)
    assert np.array_equal(got, oracle.gauss_seidel(u0, S))


@pytest.mark.parametrize("base_off", [1, 3, 6])
def test_protocol_with_other_alignments(base_off):
    """Chunk boundaries follow each line's own alignment; any array base
    offset gives the sequential result."""
    u0 = si.uniform_padded(37, 17, 12, 1, seed=base_off, lo=-1.0, hi=1.0)
    got = M.simulate(u0, 3, workers=5, seed=base_off, base_off=base_off)
    assert np.array_equal(got, oracle.gauss_seidel(u0, 3))


def test_ticket_order_is_topological():
    items = M.items_table(5, 4, 6)
    pos = {it: n for n, it in enumerate(items)}
    assert len(pos) == 5 * 4 * 6
    for (tau, J, K), n in pos.items():
        for d in ((tau, J - 1, K), (tau, J, K - 1), (tau - 1, J + 1, K), (tau - 1, J, K + 1),
                  (tau - 1, J, K)):
            if d in pos:
                assert pos[d] < n


def test_protocol_model_catches_early_publish():
    """Publishing a chunk before its stores have been issued and completed
    lets a consumer read stale values; the model must see that."""
    u0 = si.uniform_padded(100, 30, 9, 1, seed=2, lo=-1.0, hi=1.0)
    got = M.simulate(u0, 5, workers=16, seed=2, publish_lag=2)
    assert not np.array_equal(got, oracle.gauss_seidel(u0, 5))


def test_protocol_model_catches_misaligned_chunks():
    """A store side whose chunk boundaries differ from the load side's (by one
    element) publishes positions it has not stored; the model must see that."""
    u0 = si.uniform_padded(37, 17, 12, 1, seed=4, lo=-1.0, hi=1.0)
    got = M.simulate(u0, 3, workers=5, seed=4, base_off=2, store_shift_error=1)
    assert not np.array_equal(got, oracle.gauss_seidel(u0, 3))
