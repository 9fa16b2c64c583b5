"""Checks that tie the CPU oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function takes a loaded oracle library (``oracle.load(path)``)
and raises ``AssertionError`` when the oracle disagrees with the fact.  They are
run against the real oracle in ``test_oracle.py`` and against deliberately
broken copies of it in ``test_oracle_mutations.py``, which shows that a
plausible mistake (dropped term, wrong sign or index, swapped operands, wrong
update order) fails at least one of them.

Sources of truth used here (none re-types the oracle's own loops in FP):
  * closed form: on a zero-ghost grid the discrete sine mode
    sin(pi p i/(nx+1)) sin(pi q j/(ny+1)) sin(pi r k/(nz+1)) is an eigenvector
    of the Jacobi update with eigenvalue a + 2b(cos(pi p/(nx+1)) + ...);
  * harmonic fixed points: constant and linear fields are reproduced exactly
    when a + 6b = 1 and the ghosts match;
  * exact rational arithmetic (fractions.Fraction) of the Sec. 3 Jacobi and
    Gauss-Seidel definitions on tiny grids with dyadic weights and integer data,
    where every FP64 intermediate is exact;
  * Young's theorem: lexicographic Gauss-Seidel on the 7-point Laplacian
    (a consistently ordered matrix) converges asymptotically with the square
    of the Jacobi rate, cos(pi/(n+1))^2; the red-black ordering is
    consistently ordered too, so red-black Gauss-Seidel has the same rate;
  * red-black Gauss-Seidel written as two masked Jacobi half-sweeps with
    numpy slicing (red sites from old values, then black sites from the new
    red ones), independent of the oracle's loop nest;
  * defect correction: m sweeps on A e = r from e = 0 added to u0 equal m
    sweeps on u from u0 (linearity).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

import oracle

EPS64 = np.finfo(np.float64).eps
EPS32 = np.finfo(np.float32).eps


def sine_mode(nx, ny, nz, p, q, r, h=1, dtype=np.float64):
    u = np.zeros((nz + 2 * h, ny + 2 * h, nx + 2 * h))
    i = np.arange(1, nx + 1)
    j = np.arange(1, ny + 1)
    k = np.arange(1, nz + 1)
    sx = np.sin(np.pi * p * i / (nx + 1))
    sy = np.sin(np.pi * q * j / (ny + 1))
    sz = np.sin(np.pi * r * k / (nz + 1))
    u[h:h + nz, h:h + ny, h:h + nx] = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    return u.astype(dtype)


def mode_lambda(nx, ny, nz, p, q, r, a, b):
    c = (math.cos(math.pi * p / (nx + 1)) + math.cos(math.pi * q / (ny + 1))
         + math.cos(math.pi * r / (nz + 1)))
    return a + 2.0 * b * c


# --------------------------------------------------------------- Jacobi -----

def pin_jacobi_sine_decay(lib):
    """Closed form: each sweep multiplies the mode by lambda (FP64 and float)."""
    cases = [((12, 10, 9), (1, 2, 3), 0.0, 1.0 / 6.0, 30),
             ((9, 11, 7), (2, 1, 1), 0.25, 0.125, 30),
             ((16, 5, 6), (3, 1, 2), 1.0 / 3.0, 1.0 / 9.0, 25)]
    for (nx, ny, nz), (p, q, r), a, b, S in cases:
        lam = mode_lambda(nx, ny, nz, p, q, r, a, b)
        assert abs(lam) ** S >= 1e-3, "pick a mode that does not vanish"
        u0 = sine_mode(nx, ny, nz, p, q, r)
        out = oracle.jacobi(u0, S, a=a, b=b, lib=lib)
        tol = 8 * S * EPS64 * np.abs(u0).max()
        err = np.abs(out - (lam ** S) * u0).max()
        assert err <= tol, (nx, ny, nz, p, q, r, a, b, err, tol)
        out32 = oracle.jacobi(u0.astype(np.float32), S, a=a, b=b, lib=lib)
        tol32 = 8 * S * EPS32 * np.abs(u0).max()
        err32 = np.abs(out32.astype(np.float64) - (lam ** S) * u0).max()
        assert err32 <= tol32, ("f32", nx, ny, nz, err32, tol32)


def pin_fixed_points(lib):
    """Constant and linear harmonic fields are exact fixed points (a + 6b = 1)."""
    nx, ny, nz = 7, 6, 5
    k, j, i = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    fields = [np.full((nz + 2, ny + 2, nx + 2), 3.0),
              (2 * i - 3 * j + 5 * k + 1).astype(np.float64),
              (0.5 * i + 0.25 * j - 1.5 * k).astype(np.float64)]
    for u in fields:
        for a, b in ((0.25, 0.125), (0.5, 1.0 / 12.0 * 1.0)):
            if a + 6 * b != 1.0:
                continue
            for fn in (oracle.jacobi, oracle.gauss_seidel, oracle.red_black):
                out = fn(u, 6, a=a, b=b, lib=lib)
                assert np.array_equal(out, u), (fn.__name__, a, b)
                out32 = fn(u.astype(np.float32), 6, a=a, b=b, lib=lib)
                assert np.array_equal(out32, u.astype(np.float32)), (fn.__name__, "f32")
    # b = 1/6 is not dyadic: at most a couple of ulps per sweep.
    u = np.full((nz + 2, ny + 2, nx + 2), 0.7)
    for fn in (oracle.jacobi, oracle.gauss_seidel, oracle.red_black):
        out = fn(u, 10, a=0.0, b=1.0 / 6.0, lib=lib)
        assert np.abs(out - 0.7).max() <= 10 * 2 * EPS64, fn.__name__


def _frac_sweeps(u, f, a, b, g, sweeps, in_place, colors=None):
    """Sec. 3 definitions in exact rational arithmetic (order-free).  With
    colors=(0, 1) each sweep is two in-place passes over the sites whose
    (i + j + k) parity (interior coordinates from 0) is that colour."""
    nz, ny, nx = len(u) - 2, len(u[0]) - 2, len(u[0][0]) - 2
    cur = [[[Fraction(v) for v in row] for row in plane] for plane in u]
    passes = [(None, in_place)] if colors is None else [(c, True) for c in colors]
    for _ in range(sweeps):
        for color, inp in passes:
            src = cur
            dst = cur if inp else [[[v for v in row] for row in plane] for plane in cur]
            for k in range(1, nz + 1):
                for j in range(1, ny + 1):
                    for i in range(1, nx + 1):
                        if color is not None and (i + j + k - 3) % 2 != color:
                            continue
                        s = (src[k][j][i - 1] + src[k][j][i + 1] + src[k][j - 1][i]
                             + src[k][j + 1][i] + src[k - 1][j][i] + src[k + 1][j][i])
                        v = a * src[k][j][i] + b * s
                        if f is not None:
                            v += g * Fraction(f[k - 1][j - 1][i - 1])
                        dst[k][j][i] = v
            cur = dst
    return cur


def _check_frac(out, exact, mant_bits=53):
    for k, plane in enumerate(exact):
        for j, row in enumerate(plane):
            for i, v in enumerate(row):
                # the fixture is only meaningful while every value is representable
                assert abs(v.numerator).bit_length() <= mant_bits, "fixture not exact"
                assert Fraction(float(out[k, j, i])) == v, (k, j, i, float(out[k, j, i]), v)


def pin_exact_rational(lib):
    """Dyadic weights + integer data: FP64 result equals the exact rational one."""
    rng = np.random.default_rng(1234)
    nx, ny, nz = 4, 3, 5
    u = rng.integers(-8, 9, size=(nz + 2, ny + 2, nx + 2)).astype(np.float64)
    f = rng.integers(-4, 5, size=(nz, ny, nx)).astype(np.float64)
    ul = u.tolist()
    fl = f.tolist()
    for a, b, g, use_f in ((Fraction(1, 4), Fraction(1, 8), Fraction(0), False),
                           (Fraction(0), Fraction(1, 8), Fraction(1, 2), True),
                           (Fraction(-1, 2), Fraction(1, 4), Fraction(3, 4), True)):
        ff = f if use_f else None
        for in_place, fn, colors in ((False, oracle.jacobi, None), (True, oracle.gauss_seidel, None),
                                     (True, oracle.red_black, (0, 1))):
            exact = _frac_sweeps(ul, fl if use_f else None, a, b, g, 5, in_place, colors)
            out = fn(u, 5, a=float(a), b=float(b), f=ff, g=float(g), lib=lib)
            _check_frac(out, exact)


def pin_exact_rational_f32(lib):
    """Same exact check for the float functions (values stay within 24 bits)."""
    rng = np.random.default_rng(99)
    a, b, g = Fraction(1, 4), Fraction(1, 8), Fraction(1, 2)
    # Gauss-Seidel chains fresh values within a sweep, so its denominators grow
    # with the grid diagonal: keep its grid and sweep count smaller.
    for in_place, fn, (nx, ny, nz), S, colors in (
            (False, oracle.jacobi, (3, 4, 3), 3, None),
            (True, oracle.gauss_seidel, (3, 2, 2), 1, None),
            (True, oracle.red_black, (3, 3, 2), 2, (0, 1))):
        u = rng.integers(-4, 5, size=(nz + 2, ny + 2, nx + 2)).astype(np.float64)
        f = rng.integers(-2, 3, size=(nz, ny, nx)).astype(np.float64)
        exact = _frac_sweeps(u.tolist(), f.tolist(), a, b, g, S, in_place, colors)
        out = fn(u.astype(np.float32), S, a=0.25, b=0.125, f=f.astype(np.float32), g=0.5, lib=lib)
        _check_frac(out.astype(np.float64), exact, mant_bits=24)


# -------------------------------------------------------- Gauss-Seidel -----

def pin_gs_rate(lib):
    """Young: asymptotic GS factor = cos(pi/(n+1))^2; Jacobi's is cos(pi/(n+1))."""
    n = 9
    rng = np.random.default_rng(7)
    u = np.zeros((n + 2, n + 2, n + 2))
    u[1:-1, 1:-1, 1:-1] = rng.random((n, n, n))
    rho_j = math.cos(math.pi / (n + 1))
    for fn, expect in ((oracle.gauss_seidel, rho_j ** 2), (oracle.red_black, rho_j ** 2),
                       (oracle.jacobi, rho_j)):
        v = fn(u, 300 if fn is oracle.jacobi else 150, lib=lib)
        w = fn(v, 1, lib=lib)
        ratio = np.linalg.norm(w) / np.linalg.norm(v)
        assert abs(ratio - expect) < 2e-3, (fn.__name__, ratio, expect)


def pin_gs_differs_from_jacobi(lib):
    """One GS sweep must use fresh x-, y-, z- values: compare an impulse response."""
    n = 5
    u = np.zeros((n + 2, n + 2, n + 2))
    u[1, 1, 1] = 6.0  # impulse at the first interior site
    g = oracle.gauss_seidel(u, 1, a=0.0, b=1.0 / 8.0, lib=lib)
    # Lexicographic order propagates the impulse to every later site with a
    # monotone path; exact values: site (1,1,2) sees u(1,1,1)_new = 0 (it was
    # overwritten by b*sum(0) = 0) -- so the impulse is erased before use.
    assert g[1, 1, 1] == 0.0
    assert np.count_nonzero(g) == 0
    # Jacobi keeps the impulse for its neighbours.
    j = oracle.jacobi(u, 1, a=0.0, b=1.0 / 8.0, lib=lib)
    assert j[1, 1, 2] == 0.75 and j[1, 2, 1] == 0.75 and j[2, 1, 1] == 0.75
    # an impulse at a central site: its three lower neighbours see the OLD
    # value through +z/+y/+x (1 each), then the site itself sees those three
    # FRESH values through -z/-y/-x (3/8); Jacobi gives 1 to all six
    # neighbours and 0 to the site.
    u = np.zeros((n + 2, n + 2, n + 2))
    u[3, 3, 3] = 8.0
    g = oracle.gauss_seidel(u, 1, a=0.0, b=1.0 / 8.0, lib=lib)
    assert g[2, 3, 3] == 1.0 and g[3, 2, 3] == 1.0 and g[3, 3, 2] == 1.0
    assert g[3, 3, 3] == 3.0 / 8.0
    j = oracle.jacobi(u, 1, a=0.0, b=1.0 / 8.0, lib=lib)
    assert j[3, 3, 3] == 0.0
    for d in ((2, 3, 3), (4, 3, 3), (3, 2, 3), (3, 4, 3), (3, 3, 2), (3, 3, 4)):
        assert j[d] == 1.0


# ------------------------------------------------ residual, refinement -----

def pin_residual_mode(lib):
    """A u for the sine mode is (6 - 2 sum cos) u in closed form."""
    nx, ny, nz = 10, 8, 6
    u = sine_mode(nx, ny, nz, 2, 3, 1)
    mu = 6.0 - 2.0 * (math.cos(2 * math.pi / (nx + 1)) + math.cos(3 * math.pi / (ny + 1))
                      + math.cos(math.pi / (nz + 1)))
    fp = 0.5 * np.ones((nz, ny, nx))
    r, rr = oracle.residual(u, fp, lib=lib)
    expect = fp - mu * u[1:-1, 1:-1, 1:-1]
    assert np.abs(r - expect).max() <= 16 * EPS64
    assert abs(rr - float(np.sum(expect * expect))) <= 1e-12 * rr


def pin_defect_correction(lib):
    """One outer step with m FP64 inner sweeps == m plain sweeps with f'."""
    n = 10
    rng = np.random.default_rng(5)
    fp = (2 * rng.random((n, n, n)) - 1) / (n + 1) ** 2
    u0 = np.zeros((n + 2, n + 2, n + 2))
    u0[1:-1, 1:-1, 1:-1] = rng.random((n, n, n)) * 1e-3
    for method in (0, 1, 2):
        m = 12
        out, rc, outer, _ = oracle.refine(u0, fp, method=method, inner_f32=False, m=m,
                                          tol=0.0, max_outer=1, lib=lib)
        assert outer == 1 and rc == -6
        plain = oracle.smooth(method, u0, m, a=0.0, b=1.0 / 6.0, f=fp, g=1.0 / 6.0, lib=lib)
        scale = np.abs(plain).max()
        assert np.abs(out - plain).max() <= 64 * m * EPS64 * scale, method
        # float inner sweeps: equal up to float rounding of the correction
        out32, _, _, _ = oracle.refine(u0, fp, method=method, inner_f32=True, m=m,
                                       tol=0.0, max_outer=1, lib=lib)
        assert np.abs(out32 - plain).max() <= 1e-5 * scale, method
        # and the general one-step form used for serving jobs
        job = oracle.refined_job(method, u0, m, a=0.0, b=1.0 / 6.0, f=fp, g=1.0 / 6.0, lib=lib)
        assert np.abs(job - plain).max() <= 1e-5 * scale, method


def pin_manufactured_solution(lib):
    """The refinement loop converges to the known solution u* = sine(1,1,1)."""
    n = 8
    us = sine_mode(n, n, n, 1, 1, 1)
    mu = 6.0 - 6.0 * math.cos(math.pi / (n + 1))
    fp = mu * us[1:-1, 1:-1, 1:-1]
    u0 = np.zeros_like(us)
    for method in (0, 1, 2):
        for inner_f32 in (False, True):
            out, rc, outer, rel = oracle.refine(u0, fp, method=method, inner_f32=inner_f32, m=16,
                                                tol=1e-10, max_outer=400, lib=lib)
            assert rc == 0 and rel <= 1e-10, (method, inner_f32, rc, rel)
            # cond(A) ~ 12/mu < 30 bounds the error by 30 * 1e-10 relative
            assert np.abs(out - us).max() <= 30 * 1e-10 * np.abs(us).max() + 1e-15
    # GS needs about half the sweeps of Jacobi (rho_GS = rho_J^2)
    _, _, oj, _ = oracle.refine(u0, fp + 1e-3, method=0, inner_f32=False, m=8, tol=1e-10,
                                max_outer=2000, lib=lib)
    _, _, og, _ = oracle.refine(u0, fp + 1e-3, method=1, inner_f32=False, m=8, tol=1e-10,
                                max_outer=2000, lib=lib)
    assert 0.4 <= og / oj <= 0.62, (oj, og)
    # red-black has the same asymptotic factor as lexicographic GS
    _, _, orb, _ = oracle.refine(u0, fp + 1e-3, method=2, inner_f32=False, m=8, tol=1e-10,
                                 max_outer=2000, lib=lib)
    assert 0.4 <= orb / oj <= 0.62, (oj, orb)


def pin_split_invariance(lib):
    """S1 sweeps then S2 sweeps equal S1 + S2 sweeps (bit-exact)."""
    rng = np.random.default_rng(3)
    u = rng.random((8, 7, 9))
    for fn in (oracle.jacobi, oracle.gauss_seidel):
        once = fn(u, 7, lib=lib)
        twice = fn(fn(u, 3, lib=lib), 4, lib=lib)
        assert np.array_equal(once, twice), fn.__name__
        assert np.array_equal(fn(u, 0, lib=lib), u)


# -------------------------------------------- operand order, both dtypes -----
# The update rule as the library header states it (and as Sec. 3 defines the
# sweep): s = ((((x- + x+) + y-) + y+) + z-) + z+, v = (a*c) + (b*s), then
# v + (g*f).  The two references below evaluate exactly that rule in IEEE
# arithmetic of the requested dtype (numpy float64 / float32 arrays and
# scalars), independently of the oracle's loop nests: Jacobi as whole-array
# slices, Gauss-Seidel as one sequential loop over flat interior indices.

def _rule(dt, c, xm, xp, ym, yp, zm, zp, a, b, g, fv):
    s = xm + xp
    s = s + ym
    s = s + yp
    s = s + zm
    s = s + zp
    v = (dt(a) * c) + (dt(b) * s) if a != 0.0 else dt(b) * s
    if fv is not None:
        v = v + (dt(g) * fv)
    return v


def _slices_jacobi(u, S, a, b, f=None, g=0.0, h=1):
    """Two-array Jacobi sweeps with numpy slices in the dtype of u."""
    dt = u.dtype.type
    cur = u.copy()
    nz, ny, nx = (d - 2 * h for d in u.shape)
    I = (slice(h, h + nz), slice(h, h + ny), slice(h, h + nx))
    for _ in range(S):
        nxt = cur.copy()
        nxt[I] = _rule(dt, cur[I],
                       cur[h:h + nz, h:h + ny, h - 1:h + nx - 1], cur[h:h + nz, h:h + ny, h + 1:h + nx + 1],
                       cur[h:h + nz, h - 1:h + ny - 1, h:h + nx], cur[h:h + nz, h + 1:h + ny + 1, h:h + nx],
                       cur[h - 1:h + nz - 1, h:h + ny, h:h + nx], cur[h + 1:h + nz + 1, h:h + ny, h:h + nx],
                       a, b, g, f)
        cur = nxt
    return cur


def _flat_gs(u, S, a, b, f=None, g=0.0, h=1):
    """In-place Gauss-Seidel as one sequential loop over the flat interior
    indices in increasing order (numpy scalars of the dtype of u)."""
    dt = u.dtype.type
    pz, py, px = u.shape
    plane = py * px
    flat = u.copy().reshape(-1)
    ff = None if f is None else f.reshape(-1)
    for _ in range(S):
        q = 0
        for k in range(h, pz - h):
            for j in range(h, py - h):
                for i in range(h, px - h):
                    o = (k * py + j) * px + i
                    flat[o] = _rule(dt, flat[o], flat[o - 1], flat[o + 1], flat[o - px],
                                    flat[o + px], flat[o - plane], flat[o + plane], a, b, g,
                                    None if ff is None else ff[q])
                    q += 1
    return flat.reshape(u.shape)


def pin_operand_order(lib):
    """Bit-exact against the stated update rule, FP64 and float, with and
    without the centre and right-hand-side terms: pins the summation order."""
    rng = np.random.default_rng(0)
    for dt in (np.float64, np.float32):
        u = np.zeros((10, 10, 10), dtype=dt)
        u[1:-1, 1:-1, 1:-1] = (2 * rng.random((8, 8, 8)) - 1).astype(dt)
        f = (rng.random((8, 8, 8)) - 0.5).astype(dt)
        for a, b, g, ff in ((0.0, 1.0 / 6.0, 0.0, None), (0.3, 0.1, 0.25, f)):
            assert np.array_equal(oracle.gauss_seidel(u, 3, a=a, b=b, f=ff, g=g, lib=lib),
                                  _flat_gs(u, 3, a, b, ff, g)), (dt, a)
        v = rng.random((7, 8, 9)).astype(dt)
        fv = (rng.random((5, 6, 7)) - 0.5).astype(dt)
        for a, b, g, ff, S in ((0.0, 1.0 / 6.0, 0.0, None, 4), (0.3, 0.1, 0.0, None, 2),
                               (0.0, 1.0 / 6.0, 1.0 / 6.0, fv, 3)):
            assert np.array_equal(oracle.jacobi(v, S, a=a, b=b, f=ff, g=g, lib=lib),
                                  _slices_jacobi(v, S, a, b, ff, g)), (dt, a, S)


def pin_red_black_masks(lib):
    """Red-black = masked Jacobi on the red sites, then on the black sites with
    the new red values (numpy slicing in the grid's dtype, same operand order:
    bit-exact, FP64 and float), and it differs from the lexicographic sweep."""
    rng = np.random.default_rng(5)
    for dt in (np.float64, np.float32):
        for h, (nx, ny, nz), a, b, use_f in ((1, (9, 6, 7), 0.0, 1.0 / 6.0, False),
                                             (2, (5, 8, 4), 0.3, 0.11, True)):
            u = (rng.random((nz + 2 * h, ny + 2 * h, nx + 2 * h)) * 2 - 1).astype(dt)
            f = (rng.random((nz, ny, nx)) - 0.5).astype(dt) if use_f else None
            g = 0.25
            kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
            parity = (ii + jj + kk) % 2
            ref = u.copy()
            I = (slice(h, h + nz), slice(h, h + ny), slice(h, h + nx))
            for _ in range(3):
                for color in (0, 1):
                    v = _rule(dt, ref[I],
                              ref[h:h + nz, h:h + ny, h - 1:h + nx - 1],
                              ref[h:h + nz, h:h + ny, h + 1:h + nx + 1],
                              ref[h:h + nz, h - 1:h + ny - 1, h:h + nx],
                              ref[h:h + nz, h + 1:h + ny + 1, h:h + nx],
                              ref[h - 1:h + nz - 1, h:h + ny, h:h + nx],
                              ref[h + 1:h + nz + 1, h:h + ny, h:h + nx], a, b, g, f)
                    ref[I] = np.where(parity == color, v, ref[I])
            out = oracle.red_black(u, 3, a=a, b=b, f=f, g=g, h=h, lib=lib)
            assert np.array_equal(out, ref), (dt, h, a)
            assert not np.array_equal(out, oracle.gauss_seidel(u, 3, a=a, b=b, f=f, g=g, h=h,
                                                               lib=lib))


# --- multigrid transfers and V-cycle ------------------------------------------
#
# Sources of truth: the hat-function definition of trilinear interpolation
# between the points i/(n+1) and I/(nc+1), evaluated in exact rationals; the
# full-weighting stencil (1/64)[1 2 1]^3 of nested grids; the transpose
# relation R = scale * P^T; the h^2 scaling (R applied to a constant gives
# (H/h)^2); and multigrid theory: a V(2,2)-cycle with a smoothing iteration on
# the 7-point Poisson matrix contracts the residual by a factor well below 1
# that does not grow with n, and the converged iterate is the exact discrete
# solution (manufactured from a random u*).


def _hat(i, n, I, nc):
    """Exact hat function of coarse point I at fine point i: max(0, 1 - |X - I|),
    X = i (nc+1)/(n+1)."""
    X = Fraction(i * (nc + 1), n + 1)
    return max(Fraction(0), 1 - abs(X - I))


def pin_mg_levels(lib):
    ns = [512]
    while len(ns) < 12 and ns[-1] >= 3:
        ns.append(int(lib.oracle_mg_coarse_n(ns[-1])))
    assert ns == [512, 255, 127, 63, 31, 15, 7, 3, 1], ns
    assert lib.oracle_mg_levels(512, 512, 512) == 9
    assert lib.oracle_mg_levels(2, 40, 40) == 1
    assert lib.oracle_mg_levels(7, 16, 3) == 2
    # h/H: 256/513 for 512 (non-nested), exactly 1/2 for nested levels
    assert lib.oracle_mg_scale(512, 512, 512) == 256.0 / 513.0
    assert lib.oracle_mg_scale(255, 255, 255) == 0.5


def pin_mg_prolong_hat(lib):
    """P e_c for a coarse delta is the tensor product of exact hat functions
    (nested: exactly; non-nested: within the rounding of three weights)."""
    for dims, dt, tol in (((7, 7, 7), np.float64, 0.0), ((10, 8, 12), np.float64, 4 * EPS64),
                          ((9, 11, 8), np.float32, 4 * EPS32), ((15, 7, 11), np.float32, 0.0)):
        nx, ny, nz = dims
        cn = oracle.mg_coarse_dims(nx, ny, nz)
        for (I, J, K) in ((1, 1, 1), (cn[0], cn[1], cn[2]), ((cn[0] + 1) // 2, 1, cn[2])):
            ec = np.zeros((cn[2] + 2, cn[1] + 2, cn[0] + 2), dtype=dt)
            ec[K, J, I] = 1.0
            ef = np.zeros((nz + 2, ny + 2, nx + 2), dtype=dt)
            out = oracle.mg_prolong_add(ef, ec, lib=lib)
            for k in range(1, nz + 1):
                hz = _hat(k, nz, K, cn[2])
                for j in range(1, ny + 1):
                    hy = _hat(j, ny, J, cn[1])
                    for i in range(1, nx + 1):
                        ex = _hat(i, nx, I, cn[0]) * hy * hz
                        got = Fraction(float(out[k, j, i]))
                        assert abs(got - ex) <= tol * max(ex, Fraction(1, 2 ** 40)) + (
                            0 if tol == 0 else Fraction(1, 2 ** 100)), (dims, dt, (I, J, K), (k, j, i))
            assert np.all(out[0] == 0) and np.all(out[:, :, 0] == 0)  # ghosts untouched


def pin_mg_full_weighting(lib):
    """Nested levels: restriction = 4 * (1/64) [1 2 1] x [1 2 1] x [1 2 1]
    around fine point 2I; bit-exact on small integer data (every partial sum
    is exact), FP64 and float."""
    rng = np.random.default_rng(7)
    for dims in ((7, 7, 7), (15, 7, 3), (11, 15, 7)):
        nx, ny, nz = dims
        for dt in (np.float64, np.float32):
            res = rng.integers(-40, 41, size=(nz, ny, nx)).astype(dt)
            rc = oracle.mg_restrict(res, lib=lib)
            pad = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.int64)
            pad[1:-1, 1:-1, 1:-1] = res.astype(np.int64)
            cn = oracle.mg_coarse_dims(nx, ny, nz)
            w = (1, 2, 1)
            for K in range(1, cn[2] + 1):
                for J in range(1, cn[1] + 1):
                    for I in range(1, cn[0] + 1):
                        acc = 0
                        for c in range(3):
                            for b in range(3):
                                for a in range(3):
                                    acc += w[a] * w[b] * w[c] * pad[2 * K + c - 1, 2 * J + b - 1,
                                                                     2 * I + a - 1]
                        assert Fraction(float(rc[K - 1, J - 1, I - 1])) == Fraction(acc, 16), (
                            dims, dt, (I, J, K))


def pin_mg_transpose_and_scale(lib):
    """<R r, e_c> = scale <r, P e_c> for random r, e_c (non-nested, non-cubic),
    and R applied to a constant gives (H/h)^2 at coarse points whose support
    stays inside the grid."""
    rng = np.random.default_rng(11)
    for dims in ((12, 10, 9), (16, 16, 16), (15, 9, 20)):
        nx, ny, nz = dims
        cn = oracle.mg_coarse_dims(nx, ny, nz)
        r = rng.standard_normal((nz, ny, nx))
        ec = np.zeros((cn[2] + 2, cn[1] + 2, cn[0] + 2))
        ec[1:-1, 1:-1, 1:-1] = rng.standard_normal((cn[2], cn[1], cn[0]))
        scale = oracle.mg_scale(nx, ny, nz, lib=lib)
        lhs = float(np.sum(oracle.mg_restrict(r, lib=lib) * ec[1:-1, 1:-1, 1:-1]))
        pe = oracle.mg_prolong_add(np.zeros((nz + 2, ny + 2, nx + 2)), ec, lib=lib)
        rhs = scale * float(np.sum(r * pe[1:-1, 1:-1, 1:-1]))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.sqrt(r.size)), (dims, lhs, rhs)
    # nested: a constant restricts to exactly (H/h)^2 = 4 away from the boundary
    rc = oracle.mg_restrict(np.ones((15, 15, 15)), lib=lib)
    assert np.all(rc[1:-1, 1:-1, 1:-1] == 4.0), rc[2, 2, 2]
    # non-nested: scale times the product of the exact hat sums of each axis
    n = 16
    nc = oracle.mg_coarse_dims(n, n, n)[0]
    rc = oracle.mg_restrict(np.ones((n, n, n)), lib=lib)
    scale = Fraction(nc + 1, n + 1)
    hs = [sum(_hat(i, n, I, nc) for i in range(1, n + 1)) for I in range(1, nc + 1)]
    for K in range(nc):
        for J in range(nc):
            for I in range(nc):
                want = float(scale * hs[I] * hs[J] * hs[K])
                assert abs(rc[K, J, I] - want) <= 1e-14 * want, ((I, J, K), rc[K, J, I], want)


def _apply_A(u):
    """(6c - s) at interior sites of a padded grid with ghost width 1."""
    c = u[1:-1, 1:-1, 1:-1]
    s = (u[1:-1, 1:-1, :-2] + u[1:-1, 1:-1, 2:] + u[1:-1, :-2, 1:-1] + u[1:-1, 2:, 1:-1] +
         u[:-2, 1:-1, 1:-1] + u[2:, 1:-1, 1:-1])
    return 6.0 * c - s


def pin_mg_convergence(lib):
    """V(2,2) contracts the residual by <= 0.35 per cycle for every smoother,
    at n = 8 and 16 alike (no growth with n), and reaches 1e-10."""
    rng = np.random.default_rng(3)
    for n in (8, 16, 15):
        fp = (2 * rng.random((n, n, n)) - 1) / (n + 1) ** 2
        u0 = np.zeros((n + 2,) * 3)
        for sm in (0, 1, 2):
            out, rc, cyc, rel, hist = oracle.mg_solve(u0, fp, smoother=sm, inner_f32=False,
                                                      pre=2, post=2, coarse=16, tol=1e-10,
                                                      max_cycles=30, lib=lib)
            assert rc == 0 and rel <= 1e-10, (n, sm, rc, rel)
            fac = (hist[-1] / hist[1]) ** (1.0 / (len(hist) - 2))
            assert fac <= 0.35, (n, sm, fac)


def pin_mg_manufactured(lib):
    """The FP32-inner V-cycle defect correction converges to the exact
    discrete solution u* of A u* = f' (f' manufactured from a random u*)."""
    rng = np.random.default_rng(5)
    for dims in ((12, 9, 10), (15, 15, 15)):
        nx, ny, nz = dims
        us = np.zeros((nz + 2, ny + 2, nx + 2))
        us[1:-1, 1:-1, 1:-1] = rng.random((nz, ny, nx))
        fp = _apply_A(us)
        for sm, most in ((0, 32), (2, 20)):
            out, rc, cyc, rel, _ = oracle.mg_solve(np.zeros_like(us), fp, smoother=sm,
                                                   inner_f32=True, tol=1e-13, max_cycles=60,
                                                   lib=lib)
            assert rc == 0 and cyc <= most, (dims, sm, rel, cyc)  # float V-cycles contract too
            assert np.max(np.abs(out - us)) <= 1e-10, (dims, sm, np.max(np.abs(out - us)))


ALL_PINS = [pin_operand_order, pin_jacobi_sine_decay, pin_fixed_points, pin_exact_rational, pin_exact_rational_f32,
            pin_gs_rate, pin_gs_differs_from_jacobi, pin_residual_mode, pin_defect_correction,
            pin_manufactured_solution, pin_split_invariance, pin_red_black_masks, pin_mg_levels,
            pin_mg_prolong_hat, pin_mg_full_weighting, pin_mg_transpose_and_scale,
            pin_mg_convergence, pin_mg_manufactured]
