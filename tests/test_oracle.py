"""The CPU oracle against facts fixed by the paper and by mathematics (no GPU)."""
import numpy as np
import pytest

import oracle
import oracle_pins
import synthetic_inputs as si


@pytest.fixture(scope="module")
def lib():
    oracle.build(force=False)
    return oracle.load()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin, lib):
    pin(lib)


def test_numpy_slicing_jacobi_bit_exact(lib):
    u = si.uniform_padded(20, 17, 13, 1, seed=2)
    ref = u.copy()
    for _ in range(5):
        c = ref[1:-1, 1:-1, 1:-1]
        s = ref[1:-1, 1:-1, :-2] + ref[1:-1, 1:-1, 2:]
        s = s + ref[1:-1, :-2, 1:-1]
        s = s + ref[1:-1, 2:, 1:-1]
        s = s + ref[:-2, 1:-1, 1:-1]
        s = s + ref[2:, 1:-1, 1:-1]
        nxt = ref.copy()
        nxt[1:-1, 1:-1, 1:-1] = 0.25 * c + 0.125 * s
        ref = nxt
    assert np.array_equal(oracle.jacobi(u, 5, a=0.25, b=0.125, lib=lib), ref)


def test_wide_ghost_layer(lib):
    """h > 1: only the innermost ghost layer is read; outer ghosts are inert."""
    u2 = si.uniform_padded(6, 5, 4, 2, seed=4)
    u1 = u2[1:-1, 1:-1, 1:-1].copy()
    for fn in (oracle.jacobi, oracle.gauss_seidel):
        a = fn(u2, 3, h=2, lib=lib)
        b = fn(u1, 3, h=1, lib=lib)
        assert np.array_equal(a[1:-1, 1:-1, 1:-1], b)
        assert np.array_equal(a[0], u2[0])


def test_golden_fixture(lib):
    """Small stored outputs written by tests/golden/make_golden.py (oracle only)."""
    import golden_io
    for case in golden_io.load_cases():
        out = golden_io.run_case(case, lib)
        assert np.array_equal(out, case["expected"]), case["name"]


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_threaded_jacobi_baseline_matches(lib, threads):
    """The OpenMP CPU baseline only splits the k loop: same bits as the
    single-threaded loop nest for any thread count, weights and ghost width."""
    for (a, b, h) in ((0.0, 1.0 / 6.0, 1), (0.3, 0.1, 2)):
        u = si.uniform_padded(23, 19, 11, h, seed=threads, lo=-1.0, hi=1.0)
        got, used = oracle.jacobi_threads(u, 5, a=a, b=b, h=h, threads=threads, lib=lib)
        assert 1 <= used <= threads
        assert np.array_equal(got, oracle.jacobi(u, 5, a=a, b=b, h=h, lib=lib))
