"""paper_1004_1741_amd -- Python binding of libstencil (gfx950 HIP kernels).

Thin ctypes marshalling over the C ABI in include/stencil.h: every smoothing
step runs in the library's HIP kernels.  PyTorch is used only to hold device
memory and to supply the current HIP stream.  There is no CPU fallback: if
libstencil.so is missing or cannot be loaded, every call raises.

Grids are torch tensors in the padded layout (nz+2h, ny+2h, nx+2h), x
contiguous, dtype float64 or float32, on a HIP device.
"""
from __future__ import annotations

import ctypes
import pathlib

__all__ = ["lib", "jacobi", "gauss_seidel", "red_black", "residual", "refine_solve", "jacobi_plan", "jacobi_tiles",
           "sync", "gs_abort", "gs_spin_limit",
           "StencilError", "SmoothService", "ST", "LIB_PATH"]

LIB_PATH = pathlib.Path(__file__).resolve().parent / "libstencil.so"


class ST:
    OK, EINVAL, ENOMEM, EHIP, EBUSY, ENOENT, ENOCONV, ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7
    FP64, FP32 = 0, 1
    BC_KEEP, BC_CONST = 0, 1


class StencilError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (status %d): %s" % (_strerror(status), status, msg))
        self.status = status


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("halo", ctypes.c_int32)]


class Weights(ctypes.Structure):
    _fields_ = [("center", ctypes.c_double), ("neighbor", ctypes.c_double),
                ("rhs", ctypes.c_double)]


class SmoothConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int32),
                ("device", ctypes.c_int32), ("t_fuse", ctypes.c_int32),
                ("sweeps_per_iteration", ctypes.c_int32)]


class SmoothJob(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("method", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("sweeps", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("weights", Weights), ("input_host", ctypes.c_void_p),
                ("output_host", ctypes.c_void_p)]


class SmoothStats(ctypes.Structure):
    _fields_ = [("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64),
                ("footprint_bytes", ctypes.c_uint64), ("lups", ctypes.c_double),
                ("batch_id", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("t_uploaded_ns", ctypes.c_int64), ("t_computed_ns", ctypes.c_int64)]


class ServiceStats(ctypes.Structure):
    _fields_ = [("pool_bytes", ctypes.c_uint64), ("footprint_high_water", ctypes.c_uint64),
                ("footprint_now", ctypes.c_uint64), ("batches", ctypes.c_int64),
                ("jobs_done", ctypes.c_int64), ("jobs_failed", ctypes.c_int64),
                ("jobs_canceled", ctypes.c_int64), ("max_resident_seen", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None

# (name, restype, argtypes) -- every symbol declared in include/stencil.h
_P = ctypes.POINTER
_vp, _i32, _i64, _dbl, _u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
SIGNATURES = [
    ("stencil_jacobi", _i32, [_P(Grid), _i32, _vp, _vp, _vp, _P(Weights), _i32, _dbl, _i32, _i32, _vp]),
    ("stencil_jacobi_plan", _i32, [_i32, _i32, _i32, _i32, _P(_i32), _P(_i32), _i32, _P(_i32)]),
    ("stencil_jacobi_tiles", _i32, [_P(Grid), _i32, _i32, _i32, _P(_i32), _P(_i32), _P(_i32),
                                    _P(_i32)]),
    ("stencil_gs", _i32, [_P(Grid), _i32, _vp, _vp, _P(Weights), _i32, _dbl, _i32, _i32, _vp]),
    ("stencil_gs_noalloc", _i32,
     [_P(Grid), _i32, _vp, _vp, _P(Weights), _i32, _dbl, _i32, _i32, _vp]),
    ("stencil_sync", _i32, [_vp]),
    ("stencil_gs_abort", _i32, [_i32]),
    ("stencil_gs_spin_limit", _i32, [_i64]),
    ("stencil_rbgs", _i32, [_P(Grid), _i32, _vp, _vp, _vp, _P(Weights), _i32, _dbl, _i32, _i32, _vp]),
    ("stencil_residual", _i32, [_P(Grid), _vp, _vp, _vp, _P(_dbl), _vp]),
    ("stencil_refine_solve", _i32, [_P(Grid), _i32, _i32, _vp, _vp, _i32, _i32, _dbl, _i32,
                                    _P(_i32), _P(_dbl), _vp]),
    ("stencil_mg_solve", _i32, [_P(Grid), _i32, _i32, _vp, _vp, _i32, _i32, _i32, _dbl, _i32,
                                _P(_i32), _P(_dbl), _vp]),
    ("smooth_init", _i32, [_P(SmoothConfig), _P(_vp)]),
    ("smooth_submit", _i32, [_vp, _P(SmoothJob), _P(_u64)]),
    ("smooth_poll", _i32, [_vp, _u64, _P(_i32), _P(SmoothStats)]),
    ("smooth_wait_all", _i32, [_vp, _i64]),
    ("smooth_service_info", _i32, [_vp, _P(ServiceStats)]),
    ("smooth_shutdown", _i32, [_vp]),
    ("stencil_strerror", ctypes.c_char_p, [_i32]),
    ("stencil_last_error", ctypes.c_char_p, []),
    ("stencil_version", ctypes.c_char_p, []),
]


def lib():
    """Load libstencil.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise ImportError("libstencil.so not built: run __graft_entry__.build() or "
                              "python -m paper_1004_1741_amd.build")
        L = ctypes.CDLL(str(LIB_PATH))
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _strerror(status):
    try:
        return lib().stencil_strerror(status).decode()
    except Exception:  # pragma: no cover - only for messages
        return "status"


def _check(rc):
    if rc != 0:
        raise StencilError(rc, lib().stencil_last_error().decode())
    return rc


def _dims(u, halo):
    pz, py, px = u.shape
    return Grid(px - 2 * halo, py - 2 * halo, pz - 2 * halo, halo)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return ST.FP64
    if t.dtype == torch.float32:
        return ST.FP32
    raise TypeError("grids must be float64 or float32 tensors")


def _dev_ptr(t, name):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _check_rhs(u, f, halo):
    if f is None:
        return
    pz, py, px = u.shape
    if tuple(f.shape) != (pz - 2 * halo, py - 2 * halo, px - 2 * halo) or f.dtype != u.dtype:
        raise ValueError("f must be interior-only with the grid's dtype")


def jacobi(u, scratch, sweeps, a=0.0, b=1.0 / 6.0, f=None, g=0.0, t_fuse=0, halo=1,
           bc=ST.BC_KEEP, bc_value=0.0, stream=None):
    """`sweeps` Jacobi sweeps on u (result in u), t_fuse sweeps per HBM pass."""
    if scratch.shape != u.shape or scratch.dtype != u.dtype:
        raise ValueError("scratch must match u")
    _check_rhs(u, f, halo)
    grid = _dims(u, halo)
    w = Weights(a, b, g)
    _check(lib().stencil_jacobi(ctypes.byref(grid), _dtype_code(u), _dev_ptr(u, "u"),
                                _dev_ptr(scratch, "scratch"), _dev_ptr(f, "f"), ctypes.byref(w),
                                bc, bc_value, int(sweeps), int(t_fuse), _stream(stream)))
    return u


def jacobi_plan(sweeps, t_fuse=0, fp32=False, rhs=False):
    n = ctypes.c_int32(0)
    fc = ctypes.c_int32(0)
    buf = (ctypes.c_int32 * max(1, sweeps))()
    _check(lib().stencil_jacobi_plan(ST.FP32 if fp32 else ST.FP64, int(bool(rhs)), int(sweeps),
                                     int(t_fuse), ctypes.byref(n), buf, len(buf),
                                     ctypes.byref(fc)))
    return list(buf[:n.value]), bool(fc.value)


def jacobi_tiles(shape, levels, fp32=False, rhs=False, halo=1):
    """Tiling of one fused pass of `levels` levels over a padded grid of
    `shape` (pz, py, px): (tile_w, tile_h, tiles, interior_tiles)."""
    pz, py, px = shape
    grid = Grid(px - 2 * halo, py - 2 * halo, pz - 2 * halo, halo)
    out = [ctypes.c_int32(0) for _ in range(4)]
    _check(lib().stencil_jacobi_tiles(ctypes.byref(grid), ST.FP32 if fp32 else ST.FP64,
                                      int(bool(rhs)), int(levels), *[ctypes.byref(o) for o in out]))
    return tuple(o.value for o in out)


def red_black(u, scratch, sweeps, a=0.0, b=1.0 / 6.0, f=None, g=0.0, t_fuse=0, halo=1,
              bc=ST.BC_KEEP, bc_value=0.0, stream=None):
    """`sweeps` red-black Gauss-Seidel sweeps on u (result in u), t_fuse sweeps
    (1..4) per pass over memory."""
    if scratch.shape != u.shape or scratch.dtype != u.dtype:
        raise ValueError("scratch must match u")
    _check_rhs(u, f, halo)
    grid = _dims(u, halo)
    w = Weights(a, b, g)
    _check(lib().stencil_rbgs(ctypes.byref(grid), _dtype_code(u), _dev_ptr(u, "u"),
                              _dev_ptr(scratch, "scratch"), _dev_ptr(f, "f"), ctypes.byref(w),
                              bc, bc_value, int(sweeps), int(t_fuse), _stream(stream)))
    return u


def gauss_seidel(u, sweeps, a=0.0, b=1.0 / 6.0, f=None, g=0.0, t_fuse=0, halo=1,
                 bc=ST.BC_KEEP, bc_value=0.0, stream=None):
    """`sweeps` in-place lexicographic Gauss-Seidel sweeps on u."""
    _check_rhs(u, f, halo)
    grid = _dims(u, halo)
    w = Weights(a, b, g)
    _check(lib().stencil_gs(ctypes.byref(grid), _dtype_code(u), _dev_ptr(u, "u"), _dev_ptr(f, "f"),
                            ctypes.byref(w), bc, bc_value, int(sweeps), int(t_fuse),
                            _stream(stream)))
    return u


def gauss_seidel_noalloc(u, sweeps, a=0.0, b=1.0 / 6.0, f=None, g=0.0, t_fuse=0, halo=1,
                         bc=ST.BC_KEEP, bc_value=0.0, stream=None):
    """gauss_seidel through the allocation-free entry point (workspace in the
    library's static device array; calls must not overlap on one device)."""
    _check_rhs(u, f, halo)
    grid = _dims(u, halo)
    w = Weights(a, b, g)
    _check(lib().stencil_gs_noalloc(ctypes.byref(grid), _dtype_code(u), _dev_ptr(u, "u"),
                                    _dev_ptr(f, "f"), ctypes.byref(w), bc, bc_value, int(sweeps),
                                    int(t_fuse), _stream(stream)))
    return u


def _check_fp64_interior(u, t, name, halo):
    """t must be None or an FP64 interior-only array matching the grid u."""
    import torch
    if t is None:
        return
    pz, py, px = u.shape
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if tuple(t.shape) != (pz - 2 * halo, py - 2 * halo, px - 2 * halo):
        raise ValueError("%s must be interior-only, shape (nz, ny, nx)" % name)


def _check_fp64_grid(u):
    import torch
    if u.dtype != torch.float64:
        raise TypeError("u must be a float64 grid")
    if u.dim() != 3:
        raise ValueError("u must be a 3-D padded grid")


def sync(stream=None):
    """Wait for the stream; raises StencilError (EHIP) if a Gauss-Seidel
    wavefront launch on this device gave up waiting since the last sync."""
    _check(lib().stencil_sync(_stream(stream)))


def gs_abort(device=0):
    """Raise the device's wavefront abort word (cleared by sync())."""
    _check(lib().stencil_gs_abort(int(device)))


def gs_spin_limit(polls=0):
    """Polls of one wavefront wait before it gives up (0 = default)."""
    _check(lib().stencil_gs_spin_limit(int(polls)))


def residual(u, fp, r=None, halo=1, stream=None):
    """r = f' - (6c - s) (FP64); returns the deterministic sum of r^2."""
    _check_fp64_grid(u)
    _check_fp64_interior(u, fp, "fp", halo)
    _check_fp64_interior(u, r, "r", halo)
    grid = _dims(u, halo)
    out = ctypes.c_double(0.0)
    _check(lib().stencil_residual(ctypes.byref(grid), _dev_ptr(u, "u"), _dev_ptr(fp, "fp"),
                                  _dev_ptr(r, "r"), ctypes.byref(out), _stream(stream)))
    return out.value


def refine_solve(u, fp, method=0, inner_fp32=True, inner_sweeps=16, t_fuse=0, rel_tol=1e-10,
                 max_outer=100000, halo=1, stream=None, raise_on_noconv=True):
    """Solve A u = f' by FP64 defect correction around an FP32 (or FP64) smoother.

    Returns (outer_rounds, relative_residual, status)."""
    _check_fp64_grid(u)
    if fp is None:
        raise ValueError("fp is required")
    _check_fp64_interior(u, fp, "fp", halo)
    grid = _dims(u, halo)
    od = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    rc = lib().stencil_refine_solve(ctypes.byref(grid), int(method),
                                    ST.FP32 if inner_fp32 else ST.FP64, _dev_ptr(u, "u"),
                                    _dev_ptr(fp, "fp"), int(inner_sweeps), int(t_fuse),
                                    float(rel_tol), int(max_outer), ctypes.byref(od),
                                    ctypes.byref(rel), _stream(stream))
    if rc != 0 and not (rc == ST.ENOCONV and not raise_on_noconv):
        _check(rc)
    return od.value, rel.value, rc


def mg_solve(u, fp, smoother=2, inner_fp32=True, pre=2, post=2, coarse_sweeps=16,
             rel_tol=1e-10, max_cycles=100, halo=1, stream=None, raise_on_noconv=True):
    """Solve A u = f' by FP64 defect correction around one multigrid V-cycle
    per step (FP32 or FP64), with weighted Jacobi (0), Gauss-Seidel (1) or
    red-black Gauss-Seidel (2) as the smoother.

    Returns (cycles, relative_residual, status)."""
    _check_fp64_grid(u)
    if fp is None:
        raise ValueError("fp is required")
    _check_fp64_interior(u, fp, "fp", halo)
    grid = _dims(u, halo)
    cd = ctypes.c_int32(0)
    rel = ctypes.c_double(0.0)
    rc = lib().stencil_mg_solve(ctypes.byref(grid), int(smoother),
                                ST.FP32 if inner_fp32 else ST.FP64, _dev_ptr(u, "u"),
                                _dev_ptr(fp, "fp"), int(pre), int(post), int(coarse_sweeps),
                                float(rel_tol), int(max_cycles), ctypes.byref(cd),
                                ctypes.byref(rel), _stream(stream))
    if rc != 0 and not (rc == ST.ENOCONV and not raise_on_noconv):
        _check(rc)
    return cd.value, rel.value, rc


class SmoothService:
    """Continuous-batching job service (smooth_init / submit / poll / shutdown)."""

    QUEUED, RUNNING, DONE, FAILED, CANCELED = 0, 1, 2, 3, 4

    def __init__(self, hbm_budget_bytes, max_inflight=64, device=0, t_fuse=0,
                 sweeps_per_iteration=0):
        cfg = SmoothConfig(int(hbm_budget_bytes), int(max_inflight), int(device), int(t_fuse),
                           int(sweeps_per_iteration))
        self._ctx = ctypes.c_void_p(None)
        _check(lib().smooth_init(ctypes.byref(cfg), ctypes.byref(self._ctx)))
        self._keep = {}

    def submit(self, u_in, out, sweeps, method=0, precision=0, a=0.0, b=1.0 / 6.0):
        """Queue one job: u_in and out are C-contiguous float64 numpy arrays
        of shape (nz+2, ny+2, nx+2) that stay alive until the job finishes."""
        pz, py, px = u_in.shape
        job = SmoothJob(px - 2, py - 2, pz - 2, int(method), int(precision), int(sweeps), 0,
                        Weights(a, b, 0.0), u_in.ctypes.data, out.ctypes.data)
        jid = ctypes.c_uint64(0)
        _check(lib().smooth_submit(self._ctx, ctypes.byref(job), ctypes.byref(jid)))
        self._keep[jid.value] = (u_in, out)
        return jid.value

    def poll(self, job_id):
        st = ctypes.c_int32(0)
        stats = SmoothStats()
        _check(lib().smooth_poll(self._ctx, ctypes.c_uint64(job_id), ctypes.byref(st),
                                 ctypes.byref(stats)))
        return st.value, stats

    def wait_all(self, timeout_ms=-1):
        _check(lib().smooth_wait_all(self._ctx, int(timeout_ms)))

    def info(self):
        s = ServiceStats()
        _check(lib().smooth_service_info(self._ctx, ctypes.byref(s)))
        return s

    def shutdown(self):
        if self._ctx:
            _check(lib().smooth_shutdown(self._ctx))
            self._ctx = ctypes.c_void_p(None)
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.shutdown()
