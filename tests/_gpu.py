"""Helpers shared by the GPU parity tests: SoA device tensors and tolerance definitions."""

from __future__ import annotations

import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_CACHE = os.path.join(ROOT, "_build", "kernels")


def dev_soa(a, ld=None, dtype=None):
    """numpy [nc, k] -> device tensor [k, ld] (component-major, cells contiguous)."""
    import torch
    a = np.asarray(a)
    if a.ndim == 1:
        a = a[:, None]
    nc, k = a.shape
    ld = nc if ld is None else ld
    out = np.zeros((k, ld), dtype=a.dtype if dtype is None else dtype)
    out[:, :nc] = a.T
    return torch.from_numpy(out).to("cuda")


def host_aos(t, nc):
    """device tensor [k, ld] -> numpy [nc, k]."""
    return t.cpu().numpy()[:, :nc].T.copy()


def empty(k, ld, dtype="float64"):
    import torch
    return torch.full((k, ld), float("nan") if dtype == "float64" else 0,
                      dtype=getattr(torch, dtype), device="cuda")


def gpu_mechanism(name):
    from paper_2510_10005_amd import Mechanism
    from synth import mechanism_file
    import oracle
    path = mechanism_file(name)
    return Mechanism(path, KERNEL_CACHE), oracle.load_mechanism(path)


def integrated_state_error(om, got, ref):
    """Per-cell, per-component error of integrated states, relative to |ref| with floors.

    T is compared relatively; species are compared as mass fractions relative to
    max(|Y_ref|, 1e-12) (below that a species carries no information at the 1e-8 level).
    """
    rho = (ref[:, 1:] * om.W).sum(axis=1)
    Yg = got[:, 1:] * om.W / rho[:, None]
    Yr = ref[:, 1:] * om.W / rho[:, None]
    eT = np.abs(got[:, 0] - ref[:, 0]) / np.abs(ref[:, 0])
    eY = np.abs(Yg - Yr) / np.maximum(np.abs(Yr), 1e-12)
    return np.concatenate([eT[:, None], eY], axis=1)


def gradient_errors(got, ref, floor=1e-3):
    """Errors of gradient arrays [cells, k]: (largest error relative to each column's largest
    |ref|, largest element-wise relative error over the entries with |ref| >= floor x that column
    maximum)."""
    scale = np.abs(ref).max(axis=0, keepdims=True)
    scale = np.where(scale > 0, scale, 1.0)
    col = (np.abs(got - ref) / scale).max()
    big = np.abs(ref) >= floor * scale
    elem = (np.abs(got - ref)[big] / np.abs(ref)[big]).max() if big.any() else 0.0
    return float(col), float(elem)
