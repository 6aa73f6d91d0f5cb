"""MoDL unrolled network (MoDL subsection, eq. update_modl) in FP64.

    x^0     = A^H y
    x^{t+1} = (A^H A + lambda I)^{-1} (A^H y + lambda D_W(x^t)),  t = 0..T-1,

with weights shared across the T unrolls and the inverse applied by CG
(``oracle.cg``).  The reverse-mode pass runs the unrolls backwards; each data
consistency block is differentiated as described in ``cg.cg_dc_backward`` (a
second CG solve on the self-adjoint operator), and the denoiser by
``cnn.denoise_backward``.  The oracle stores every state; it does not
recompute (the paper's checkpointing container trades memory for recompute,
which does not change the result).

Loss (eq. network_optimize with the MSE loss of the nn-library): the mean over
all B*H*W complex pixels of |x^T - x_ref|^2.  Its DF^H(1) gradient is
2 (x^T - x_ref) / (B H W).
"""
from __future__ import annotations

import numpy as np

from . import cg, cnn


def forward(aHy, S, m, weights, lam, T, n_cg, bf16=False):
    """Returns (x^T, states [x^0..x^T], zs [z^0..z^{T-1}]).
    bf16: denoiser operands rounded to bfloat16 (see oracle.cnn)."""
    x = np.asarray(aHy, dtype=np.complex128)
    states, zs = [x], []
    for _ in range(T):
        z = cnn.denoise(x, weights, bf16=bf16)
        x, _ = cg.cg_dc(aHy, z, S, m, lam, n_cg)
        zs.append(z)
        states.append(x)
    return x, states, zs


def backward(g_out, states, zs, aHy, S, m, weights, lam, T, n_cg, bf16=False):
    """Reverse mode.  Returns (grads [(gW, gb)], g_lambda [B], g_aHy)."""
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    g = np.asarray(g_out, dtype=np.complex128)
    gW = [(np.zeros_like(np.asarray(W, dtype=np.float64)),
           np.zeros_like(np.asarray(b, dtype=np.float64))) for W, b in weights]
    g_lam = np.zeros(lam.shape)
    g_a = np.zeros_like(g)
    for t in range(T - 1, -1, -1):
        v, g_z, gl = cg.cg_dc_backward(g, states[t + 1], zs[t], S, m, lam, n_cg)
        g_lam += gl
        g_a += v
        g, lg = cnn.denoise_backward(states[t], weights, g_z, bf16=bf16)
        gW = [(a[0] + b[0], a[1] + b[1]) for a, b in zip(gW, lg)]
    g_a += g  # x^0 = A^H y
    return gW, g_lam, g_a


def mse(x, ref):
    d = np.asarray(x, dtype=np.complex128) - np.asarray(ref, dtype=np.complex128)
    return float(np.mean(np.abs(d) ** 2))


def mse_grad(x, ref):
    d = np.asarray(x, dtype=np.complex128) - np.asarray(ref, dtype=np.complex128)
    return 2.0 * d / d.size
