"""The paper's own multicore schemes on the host CPU (FP64, POSIX threads).

A CPU baseline to report next to the GPU library, comparable with the paper's
x86 numbers: the temporal wavefront Jacobi of Sec. 4 (thread groups, one
sweep per thread, two planes apart, a spin barrier after every plane, skewed
y-blocks joined by boundary arrays) and the pipeline-parallel lexicographic
Gauss-Seidel of Sec. 3 combined with the Sec. 4 wavefront.  The arithmetic is
in ``wavefront.c``; this module builds it and calls it through ctypes.  It
shares no code with the GPU library or with the test oracle.  Grids use the
padded layout of ``synthetic_inputs`` (ghost layer of width h, x contiguous);
inputs are copied, never modified.
"""
from __future__ import annotations

import ctypes
import os
import pathlib
import subprocess

import numpy as np

_HERE = pathlib.Path(__file__).resolve().parent
_SRC = _HERE / "wavefront.c"
_LIB_PATH = _HERE / "libwavefront.so"
CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fno-fast-math", "-fno-unsafe-math-optimizations",
          "-pthread", "-fPIC", "-shared", "-std=c11"]

_lib = None


def build(force: bool = True):
    """Compile wavefront.c with gcc (no FMA contraction, IEEE semantics)."""
    if _LIB_PATH.exists() and not force and _LIB_PATH.stat().st_mtime >= _SRC.stat().st_mtime:
        return _LIB_PATH
    tmp = _LIB_PATH.with_suffix(".so.tmp%d" % os.getpid())
    subprocess.run(["gcc", *CFLAGS, "-o", str(tmp), str(_SRC)], check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = ctypes.CDLL(str(_LIB_PATH))
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        lib.wf_jacobi_f64.argtypes = [i64, i64, i64, i64, vp, vp, vp, dbl, dbl, dbl, i32, i32,
                                      i32, i64]
        lib.wf_jacobi_f64.restype = i32
        lib.wf_gs_f64.argtypes = [i64, i64, i64, i64, vp, vp, dbl, dbl, dbl, i32, i32, i32]
        lib.wf_gs_f64.restype = i32
        lib.wf_cpu_count.argtypes = []
        lib.wf_cpu_count.restype = i32
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _prep(u, h, f):
    out = np.ascontiguousarray(u, dtype=np.float64).copy()
    pz, py, px = out.shape
    nx, ny, nz = px - 2 * h, py - 2 * h, pz - 2 * h
    fa = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
    if fa is not None and fa.shape != (nz, ny, nx):
        raise ValueError("f must be interior-only with shape (nz, ny, nx)")
    return out, fa, nx, ny, nz


def _check(rc):
    if rc == -1:
        raise ValueError("invalid arguments")
    if rc == -2:
        raise MemoryError("allocation failed")
    if rc != 0:
        raise RuntimeError("threads could not be started (%d)" % rc)


def cpu_count() -> int:
    """Threads this process may run on (its CPU affinity set)."""
    return int(load().wf_cpu_count())


def jacobi(u, sweeps, t=4, groups=1, block_y=16, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1,
           scratch=None):
    """`sweeps` Jacobi sweeps by the temporal wavefront: t threads per group
    (one sweep each), `groups` thread groups on consecutive y-blocks of about
    `block_y` rows.  Uses t * groups threads.  Returns the new grid."""
    out, fa, nx, ny, nz = _prep(u, h, f)
    if scratch is None or scratch.shape != out.shape or scratch.dtype != np.float64:
        scratch = np.empty_like(out)
    _check(load().wf_jacobi_f64(nx, ny, nz, h, _ptr(out), _ptr(scratch), _ptr(fa), float(a),
                                float(b), float(g), int(sweeps), int(t), int(groups),
                                int(block_y)))
    return out


def gauss_seidel(u, sweeps, t=4, subblocks=4, a=0.0, b=1.0 / 6.0, f=None, g=0.0, h=1):
    """`sweeps` lexicographic Gauss-Seidel sweeps: t sweeps in flight, each
    pipelined over `subblocks` row blocks of a plane (t * subblocks threads;
    t = 1 is the plain pipeline-parallel scheme).  Returns the new grid."""
    out, fa, nx, ny, nz = _prep(u, h, f)
    _check(load().wf_gs_f64(nx, ny, nz, h, _ptr(out), _ptr(fa), float(a), float(b), float(g),
                            int(sweeps), int(t), int(subblocks)))
    return out
