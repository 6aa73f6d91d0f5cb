"""Error measures used to compare results.

rel_err(a, ref) = ||a - ref||_2 / ||ref||_2 over the whole array (operator
parity); nrmse is the same quantity used as an image-quality figure against
the phantom.  The paper's foreground-masked PSNR/SSIM needs a coil foreground
that the synthetic coils (sum |S|^2 = 1 everywhere) do not have, so the plain
L2 ratio is used.
"""
from __future__ import annotations

import numpy as np


def rel_err(a, ref):
    a = np.asarray(a).astype(np.complex128)
    ref = np.asarray(ref).astype(np.complex128)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((a - ref).ravel()) / (den if den > 0 else 1.0))


def nrmse(x, ref):
    return rel_err(x, ref)


def nrmse_per_slice(x, ref):
    x = np.asarray(x).astype(np.complex128)
    ref = np.asarray(ref).astype(np.complex128)
    return np.array([rel_err(x[b], ref[b]) for b in range(x.shape[0])])
