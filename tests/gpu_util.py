"""Helpers for the GPU parity tests (device transfers, cropping for sampled checks)."""
import sys

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device (torch.cuda.is_available() is False)")
    return torch


def to_dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()


def say(*msg):
    print(*msg, flush=True)
    sys.stdout.flush()


def assert_same(gpu, ref, what):
    """Bit-exact by value (+0 == -0), with a readable report on mismatch."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    bad = gpu != ref
    if bad.any():
        idx = np.argwhere(bad)
        k = tuple(idx[0])
        diff = np.abs(gpu.astype(np.float64) - ref.astype(np.float64))
        raise AssertionError("%s: %d of %d values differ; first at %s gpu=%r ref=%r; max |diff|=%g"
                             % (what, bad.sum(), bad.size, k, gpu[k], ref[k], diff.max()))


def crop_for_sample(u, center, sweeps, h=1, margin=None):
    """Sub-box of padded grid u whose centre sites are unaffected, after `sweeps`
    Jacobi sweeps, by freezing the box's outer layer.  A Jacobi sweep moves
    information one site, so a site at distance > sweeps from every cut face
    sees exactly the full-grid evolution.  Returns (sub, slices, inner) where
    inner indexes the exact region inside sub."""
    m = sweeps + 1 if margin is None else margin
    sl, inner = [], []
    for ax, c in enumerate(center):
        n = u.shape[ax]
        lo = max(0, c - m)
        hi = min(n, c + m + 1)
        sl.append(slice(lo, hi))
        inner.append(c - lo)
    return np.ascontiguousarray(u[tuple(sl)]), tuple(sl), tuple(inner)
