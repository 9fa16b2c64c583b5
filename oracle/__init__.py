"""CPU oracle for the iterated 3D 7-point smoothers -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and must never serve as a fallback for it.

The arithmetic lives in ``oracle.c`` (plain C loops, FP64 unless a function
says float); this module only builds and calls it through ctypes.  Every
function takes and returns numpy arrays in the padded layout described in
``synthetic_inputs``; inputs are copied, never modified.
"""
from __future__ import annotations

import ctypes
import os
import pathlib
import subprocess

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB_PATH = _HERE / "liboracle.so"
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
          "-fopenmp", "-fPIC", "-shared", "-std=c11"]

_lib = None


def build(force: bool = True, out: pathlib.Path | None = None, src: pathlib.Path | None = None):
    """Compile the oracle with gcc (no FMA contraction, IEEE semantics)."""
    out = pathlib.Path(out) if out else _LIB_PATH
    src = pathlib.Path(src) if src else _SRC
    if out.exists() and not force and out.stat().st_mtime >= src.stat().st_mtime:
        return out
    tmp = out.with_suffix(".so.tmp%d" % os.getpid())
    subprocess.run(["gcc", *CFLAGS, "-o", str(tmp), str(src), "-lm"], check=True)
    os.replace(tmp, out)
    return out


def load(path: pathlib.Path | None = None):
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(str(path)))
    if _lib is None:
        build(force=False)
        _lib = _bind(ctypes.CDLL(str(_LIB_PATH)))
    return _lib


def _bind(lib):
    i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    for name in ("oracle_jacobi_f64", "oracle_gs_f64", "oracle_jacobi_f32", "oracle_gs_f32",
                 "oracle_rbgs_f64", "oracle_rbgs_f32"):
        fn = getattr(lib, name)
        fn.argtypes = [i64, i64, i64, i64, vp, vp, dbl, dbl, dbl, i32]
        fn.restype = i32
    lib.oracle_jacobi_f64_threads.argtypes = [i64, i64, i64, i64, vp, dbl, dbl, i32, i32]
    lib.oracle_jacobi_f64_threads.restype = i32
    lib.oracle_sumsq.argtypes = [vp, i64]
    lib.oracle_sumsq.restype = dbl
    lib.oracle_residual_f64.argtypes = [i64, i64, i64, i64, vp, vp, vp]
    lib.oracle_residual_f64.restype = dbl
    lib.oracle_defect_f64.argtypes = [i64, i64, i64, i64, vp, vp, dbl, dbl, dbl, vp]
    lib.oracle_defect_f64.restype = i32
    lib.oracle_refine.argtypes = [i64, i64, i64, i64, i32, vp, vp, i32, i32, dbl, i32,
                                  ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    lib.oracle_refine.restype = i32
    lib.oracle_refined_job.argtypes = [i64, i64, i64, i64, i32, vp, vp, dbl, dbl, dbl, i32]
    lib.oracle_refined_job.restype = i32
    for name in ("oracle_mg_restrict_f64", "oracle_mg_restrict_f32"):
        getattr(lib, name).argtypes = [i64, i64, i64, vp, vp, dbl]
        getattr(lib, name).restype = None
    for name in ("oracle_mg_prolong_add_f64", "oracle_mg_prolong_add_f32"):
        getattr(lib, name).argtypes = [i64, i64, i64, i64, vp, vp]
        getattr(lib, name).restype = None
    lib.oracle_mg_residual_f32.argtypes = [i64, i64, i64, i64, vp, vp, vp]
    lib.oracle_mg_residual_f32.restype = None
    lib.oracle_mg_levels.argtypes = [i64, i64, i64]
    lib.oracle_mg_levels.restype = i32
    lib.oracle_mg_coarse_n.argtypes = [i64]
    lib.oracle_mg_coarse_n.restype = i64
    lib.oracle_mg_scale.argtypes = [i64, i64, i64]
    lib.oracle_mg_scale.restype = dbl
    lib.oracle_mg_solve.argtypes = [i64, i64, i64, i64, i32, i32, vp, vp, i32, i32, i32, dbl, i32,
                                    ctypes.POINTER(i32), ctypes.POINTER(dbl), vp]
    lib.oracle_mg_solve.restype = i32
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dims(u, h):
    pz, py, px = u.shape
    return px - 2 * h, py - 2 * h, pz - 2 * h


def _smooth(kind, u, h, f, a, b, g, sweeps, lib):
    lib = lib or load()
    dt = np.float32 if kind.endswith("f32") else np.float64
    out = np.ascontiguousarray(u, dtype=dt).copy()
    fa = None if f is None else np.ascontiguousarray(f, dtype=dt)
    nx, ny, nz = _dims(out, h)
    if fa is not None and fa.shape != (nz, ny, nx):
        raise ValueError("f must be interior-only with shape (nz, ny, nx)")
    rc = getattr(lib, "oracle_" + kind)(nx, ny, nz, h, _ptr(out), _ptr(fa), float(a),
                                        float(b), float(g), int(sweeps))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return out


def jacobi(u, sweeps, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1, lib=None):
    """`sweeps` two-array Jacobi sweeps (FP64 if u is float64, else float)."""
    kind = "jacobi_f32" if np.asarray(u).dtype == np.float32 else "jacobi_f64"
    return _smooth(kind, u, h, f, a, b, g, sweeps, lib)


def gauss_seidel(u, sweeps, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1, lib=None):
    """`sweeps` in-place lexicographic Gauss-Seidel sweeps."""
    kind = "gs_f32" if np.asarray(u).dtype == np.float32 else "gs_f64"
    return _smooth(kind, u, h, f, a, b, g, sweeps, lib)


def jacobi_threads(u, sweeps, a=0.0, b=1.0 / 6.0, h=1, threads=0, lib=None):
    """The FP64 Jacobi loops with the k loop on OpenMP threads (CPU baseline;
    same result as `jacobi`).  Returns (result, threads used)."""
    lib = lib or load()
    out = np.ascontiguousarray(u, dtype=np.float64).copy()
    nx, ny, nz = _dims(out, h)
    used = lib.oracle_jacobi_f64_threads(nx, ny, nz, h, _ptr(out), float(a), float(b),
                                         int(sweeps), int(threads))
    if used < 1:
        raise MemoryError("oracle allocation failed")
    return out, used


def red_black(u, sweeps, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1, lib=None):
    """`sweeps` in-place red-black Gauss-Seidel sweeps (red: i + j + k even)."""
    kind = "rbgs_f32" if np.asarray(u).dtype == np.float32 else "rbgs_f64"
    return _smooth(kind, u, h, f, a, b, g, sweeps, lib)


def smooth(method, u, sweeps, **kw):
    return (jacobi, gauss_seidel, red_black)[method](u, sweeps, **kw)


def residual(u, fp, h=1, lib=None):
    """r = f' - (6c - s) (interior-only) and the sequential sum of r^2."""
    lib = lib or load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    nx, ny, nz = _dims(u, h)
    fpa = None if fp is None else np.ascontiguousarray(fp, dtype=np.float64)
    r = np.empty((nz, ny, nx))
    rr = lib.oracle_residual_f64(nx, ny, nz, h, _ptr(u), _ptr(fpa), _ptr(r))
    return r, rr


def sumsq(x, lib=None):
    lib = lib or load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    return lib.oracle_sumsq(_ptr(x), x.size)


def defect(u, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1, lib=None):
    """(one update of u) - u, interior-only, FP64."""
    lib = lib or load()
    u = np.ascontiguousarray(u, dtype=np.float64)
    nx, ny, nz = _dims(u, h)
    fa = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
    r = np.empty((nz, ny, nx))
    lib.oracle_defect_f64(nx, ny, nz, h, _ptr(u), _ptr(fa), float(a), float(b), float(g), _ptr(r))
    return r


def refine(u, fp, method=0, inner_f32=True, m=16, tol=1e-10, max_outer=1000, h=1, lib=None):
    """Defect-correction solve of A u = f'; returns (u, status, outer, rel)."""
    lib = lib or load()
    out = np.ascontiguousarray(u, dtype=np.float64).copy()
    fpa = np.ascontiguousarray(fp, dtype=np.float64)
    nx, ny, nz = _dims(out, h)
    od = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = lib.oracle_refine(nx, ny, nz, h, int(method), _ptr(out), _ptr(fpa), int(bool(inner_f32)),
                           int(m), float(tol), int(max_outer), ctypes.byref(od), ctypes.byref(rel))
    if rc == -2:
        raise MemoryError("oracle allocation failed")
    return out, rc, od.value, rel.value


def refined_job(method, u, sweeps, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1, lib=None):
    """One defect-correction step with float inner sweeps (see oracle.c)."""
    lib = lib or load()
    out = np.ascontiguousarray(u, dtype=np.float64).copy()
    fa = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
    nx, ny, nz = _dims(out, h)
    rc = lib.oracle_refined_job(nx, ny, nz, h, int(method), _ptr(out), _ptr(fa), float(a),
                                float(b), float(g), int(sweeps))
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return out


# --- multigrid (test infrastructure like everything here) -------------------

def mg_coarse_dims(nx, ny, nz):
    """Interior extents of the next coarser level: floor((n+1)/2) - 1 per axis."""
    return (nx + 1) // 2 - 1, (ny + 1) // 2 - 1, (nz + 1) // 2 - 1


def mg_scale(nx, ny, nz, lib=None):
    """h/H factor of the restriction from this level to the next (FP64)."""
    lib = lib or load()
    return float(lib.oracle_mg_scale(nx, ny, nz))


def mg_levels(nx, ny, nz, lib=None):
    lib = lib or load()
    return int(lib.oracle_mg_levels(nx, ny, nz))


def mg_restrict(res, scale=None, lib=None):
    """scale * P^T res for an interior-only fine residual (scale defaults to
    the level's h/H, as in the V-cycle)."""
    lib = lib or load()
    dt = np.float32 if np.asarray(res).dtype == np.float32 else np.float64
    res = np.ascontiguousarray(res, dtype=dt)
    fnz, fny, fnx = res.shape
    cnx, cny, cnz = mg_coarse_dims(fnx, fny, fnz)
    if scale is None:
        scale = mg_scale(fnx, fny, fnz, lib)
    rc = np.zeros((cnz, cny, cnx), dtype=dt)
    fn = lib.oracle_mg_restrict_f32 if dt == np.float32 else lib.oracle_mg_restrict_f64
    fn(fnx, fny, fnz, _ptr(res), _ptr(rc), float(scale))
    return rc


def mg_prolong_add(ef, ec, h=1, lib=None):
    """ef + P ec: trilinear interpolation of the padded coarse correction ec
    (ghost width 1) added to the padded fine correction ef (ghost width h)."""
    lib = lib or load()
    dt = np.float32 if np.asarray(ef).dtype == np.float32 else np.float64
    out = np.ascontiguousarray(ef, dtype=dt).copy()
    ec = np.ascontiguousarray(ec, dtype=dt)
    fnx, fny, fnz = _dims(out, h)
    if ec.shape != tuple(d + 2 for d in mg_coarse_dims(fnz, fny, fnx)):
        raise ValueError("coarse grid does not match the fine grid")
    fn = lib.oracle_mg_prolong_add_f32 if dt == np.float32 else lib.oracle_mg_prolong_add_f64
    fn(fnx, fny, fnz, h, _ptr(out), _ptr(ec))
    return out


def mg_solve(u, fp, smoother=2, inner_f32=True, pre=2, post=2, coarse=16, tol=1e-10,
             max_cycles=50, h=1, lib=None):
    """Multigrid-preconditioned defect correction (see oracle.c); returns
    (u, status, cycles, rel, history of relative residuals)."""
    lib = lib or load()
    out = np.ascontiguousarray(u, dtype=np.float64).copy()
    fpa = np.ascontiguousarray(fp, dtype=np.float64)
    nx, ny, nz = _dims(out, h)
    if fpa.shape != (nz, ny, nx):
        raise ValueError("fp must be interior-only with shape (nz, ny, nx)")
    hist = np.full(max_cycles + 1, np.nan)
    cd = ctypes.c_int(0)
    rel = ctypes.c_double(0.0)
    rc = lib.oracle_mg_solve(nx, ny, nz, h, int(smoother), int(bool(inner_f32)), _ptr(out),
                             _ptr(fpa), int(pre), int(post), int(coarse), float(tol),
                             int(max_cycles), ctypes.byref(cd), ctypes.byref(rel), _ptr(hist))
    if rc == -2:
        raise MemoryError("oracle allocation failed")
    return out, rc, cd.value, rel.value, hist[:cd.value + 1]
