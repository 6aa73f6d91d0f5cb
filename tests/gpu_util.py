"""Helpers shared by the GPU tests (moving seeded inputs to the device,
packing uneven batches, error measures)."""
import numpy as np
import torch

from synthetic import batch_inputs, slice_inputs


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel(a, ref):
    a = np.asarray(a).astype(np.complex128).ravel()
    ref = np.asarray(ref).astype(np.complex128).ravel()
    return float(np.linalg.norm(a - ref) / max(np.linalg.norm(ref), 1e-300))


def inputs(seeds, H, W, C, R=4, nc=None, kind="vd"):
    nc = nc if nc is not None else max(2, min(24, H // 8))
    return batch_inputs(seeds, H, W, C, R, nc, kind)


def uneven(shapes, seed0=5000, R=4, kind="vd"):
    """Per-slice inputs for shapes [(H, W, C), ...] plus packed flat arrays."""
    sl = [slice_inputs(seed0 + i, H, W, C, R, max(2, min(24, H // 8)), kind)
          for i, (H, W, C) in enumerate(shapes)]
    packed = {k: np.concatenate([s[k].ravel() for s in sl]) for k in sl[0]}
    return sl, packed


def maxrel(a, ref):
    """Largest element error relative to the largest reference magnitude."""
    a = np.asarray(a).astype(np.complex128).ravel()
    ref = np.asarray(ref).astype(np.complex128).ravel()
    return float(np.max(np.abs(a - ref)) / max(np.max(np.abs(ref)), 1e-300))


def oracle_threads():
    """Context in which the FP64 oracle's FFTs use every host core (its BLAS
    calls already do)."""
    import os

    import scipy.fft
    return scipy.fft.set_workers(min(16, os.cpu_count() or 1))
