"""Seeded synthetic inputs for the 3D 7-point smoother workloads.

This module only draws random numbers and lays them out; it holds none of the
smoother's arithmetic.  Both the CPU oracle (under ``oracle/``) and the GPU
library are fed from here, so the two sides see byte-identical inputs.

Layout convention (shared by every consumer): a grid with interior extents
``nx, ny, nz`` and a ghost layer of width ``h`` is a C-ordered array of shape
``(nz + 2h, ny + 2h, nx + 2h)``; x is the contiguous axis.  Ghost cells hold
Dirichlet boundary values.

Recipes (the workloads of the paper's Sec. 3 and Sec. 4 experiments, scaled to
the sizes this library is measured on):

* uniform fill: ``numpy.random.default_rng(seed).random(padded_shape)`` fills
  the whole padded array (interior and ghost cells) in C order; ``[-1, 1)`` is
  ``2*U - 1``.  Ghost cells are then either kept or overwritten with a constant.
* right-hand side: ``2*default_rng(seed).random((nz, ny, nx)) - 1`` (interior
  only).
* serving stream: exponential inter-arrival gaps, per-job extents uniform in
  ``[32, 256]``, method and precision Bernoulli(1/2), sweeps uniform in
  ``[2, 20]``, job input drawn from ``default_rng([seed, job])``.
"""
from __future__ import annotations

import dataclasses

import numpy as np


def padded_shape(nx: int, ny: int, nz: int, h: int = 1) -> tuple:
    return (nz + 2 * h, ny + 2 * h, nx + 2 * h)


def uniform_padded(nx, ny, nz, h=1, seed=0, lo=0.0, hi=1.0, dtype=np.float64):
    """Padded grid filled with U[lo, hi) from ``default_rng(seed)`` (C order)."""
    rng = np.random.default_rng(seed)
    a = rng.random(padded_shape(nx, ny, nz, h))
    if (lo, hi) == (-1.0, 1.0):
        a = 2.0 * a - 1.0
    elif (lo, hi) != (0.0, 1.0):
        a = lo + (hi - lo) * a
    return np.ascontiguousarray(a.astype(dtype))


def set_ghosts(a: np.ndarray, h: int, value: float) -> np.ndarray:
    """Overwrite every ghost cell of padded array ``a`` with ``value`` (in place)."""
    a[:h, :, :] = value
    a[-h:, :, :] = value
    a[:, :h, :] = value
    a[:, -h:, :] = value
    a[:, :, :h] = value
    a[:, :, -h:] = value
    return a


def interior(a: np.ndarray, h: int = 1) -> np.ndarray:
    return a[h:-h, h:-h, h:-h]


def uniform_rhs(nx, ny, nz, seed=0, dtype=np.float64):
    """Interior-only right-hand side, U[-1, 1) from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray((2.0 * rng.random((nz, ny, nx)) - 1.0).astype(dtype))


# --- the named workloads ------------------------------------------------------

def jacobi_small(seed=0):
    """64^3 interior, ghost value 0, interior U[0,1); a=0, b=1/6; 10 sweeps."""
    u = set_ghosts(uniform_padded(64, 64, 64, 1, seed), 1, 0.0)
    return dict(nx=64, ny=64, nz=64, h=1, u=u, a=0.0, b=1.0 / 6.0, sweeps=10)


def jacobi_512(seed=0, n=512):
    """512^3 interior; ghost and interior both U[0,1) (one draw); 100 sweeps."""
    u = uniform_padded(n, n, n, 1, seed)
    return dict(nx=n, ny=n, nz=n, h=1, u=u, a=0.0, b=1.0 / 6.0, sweeps=100)


def gs_384(seed=0, n=384):
    """384^3 interior, ghost value 0, interior U[-1,1); a=0, b=1/6; 50 sweeps."""
    u = set_ghosts(uniform_padded(n, n, n, 1, seed, -1.0, 1.0), 1, 0.0)
    return dict(nx=n, ny=n, nz=n, h=1, u=u, a=0.0, b=1.0 / 6.0, sweeps=50)


def poisson(n=512, seed=0):
    """-Laplace(u) = f on the unit cube, h = 1/(n+1), f U[-1,1), u0 = 0, zero ghosts."""
    f = uniform_rhs(n, n, n, seed)
    u = np.zeros(padded_shape(n, n, n, 1))
    return dict(nx=n, ny=n, nz=n, h=1, u=u, f=f)


@dataclasses.dataclass
class ServingJob:
    job: int
    arrival_s: float
    nx: int
    ny: int
    nz: int
    method: int        # 0 = Jacobi, 1 = Gauss-Seidel
    sweeps: int
    precision: int     # 0 = FP64, 1 = FP32-refined
    seed: tuple

    def make_input(self) -> np.ndarray:
        rng = np.random.default_rng(list(self.seed))
        return np.ascontiguousarray(rng.random(padded_shape(self.nx, self.ny, self.nz, 1)))


def serving_stream(n_jobs=2000, rate_per_s=100.0, seed=0, dim_lo=32, dim_hi=256,
                   sweeps_lo=2, sweeps_hi=20):
    """Poisson arrival process of smoothing jobs with uneven, non-cubic grids."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_jobs)
    t = np.cumsum(gaps) - gaps[0]
    dims = rng.integers(dim_lo, dim_hi + 1, size=(n_jobs, 3))
    method = rng.integers(0, 2, size=n_jobs)
    sweeps = rng.integers(sweeps_lo, sweeps_hi + 1, size=n_jobs)
    prec = rng.integers(0, 2, size=n_jobs)
    return [ServingJob(job=i, arrival_s=float(t[i]), nx=int(dims[i, 0]), ny=int(dims[i, 1]),
                       nz=int(dims[i, 2]), method=int(method[i]), sweeps=int(sweeps[i]),
                       precision=int(prec[i]), seed=(seed, i))
            for i in range(n_jobs)]
