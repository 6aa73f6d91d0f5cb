"""Soft-SENSE: the SENSE model with several sets of coil sensitivity maps
(Extensions to the SENSE-Model subsection), in FP64.  Test infrastructure
only: nothing in the product imports this module.

With M map sets the image has one component per set, x = (x_1, ..., x_M),
and the forward operator adds the sets before the Fourier transform:

    y_c = P F (sum_m S_{m,c} x_m),        (A^H y)_m = sum_c conj(S_{m,c}) F^H P^H y_c.

M = 1 is the SENSE operator of oracle.sense.  In the networks only the
image of the first set is updated by the network block (MoDL: the denoiser
acts on x_1, the other sets pass unchanged into the data-consistency block),
and the training loss is the MSE on the coil images sum_m S_{m,c} x_m.

Shapes: x [B, M, H, W], S [B, M, C, H, W], m [B, H], y [B, C, H, W].
Readings: as oracle.sense (centered unitary F, binary row mask); the soft
image is a vector of M H W entries per slice for CG's inner products.
"""
from __future__ import annotations

import numpy as np

from . import cg as ocg
from . import cnn
from . import sense


def _c(a):
    return np.asarray(a).astype(np.complex128)


def coil_images(x, S):
    """sum_m S_{m,c} x_m: [B, C, H, W]."""
    return np.sum(_c(S) * _c(x)[:, :, None], axis=1)


def soft_fwd(x, S, m):
    return sense._rowmask(m) * sense.fft2c(coil_images(x, S))


def soft_adj(y, S, m):
    u = sense.ifft2c(sense._rowmask(m) * _c(y))  # [B, C, H, W]
    return np.sum(np.conj(_c(S)) * u[:, None], axis=2)


def soft_normal(x, S, m, lam):
    lam = np.asarray(lam, dtype=np.float64).reshape(-1, 1, 1, 1)
    return soft_adj(soft_fwd(x, S, m), S, m) + lam * _c(x)


def soft_measure(x, S, m, noise):
    """Noisy sampled k-space of the soft model (noise added on sampled rows)."""
    return sense._rowmask(m) * (sense.fft2c(coil_images(x, S)) + _c(noise))


def _flat(x):
    B, M, H, W = x.shape
    return x.reshape(B, M * H, W)


def soft_cg_dc(aHy, z, S, m, lam, n_iter):
    """x = (A^H A + lambda I)^{-1} (A^H y + lambda z) for the soft operator by
    n_iter CG steps from 0 (the CG of oracle.cg on the M H W-entry vector of
    each slice).  z = None means 0."""
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    b = _c(aHy)
    shape = b.shape
    if z is not None:
        b = b + lam[:, None, None, None] * _c(z)
    op = lambda v: _flat(soft_normal(v.reshape(shape), S, m, lam))
    x, hist = ocg.cg(op, _flat(b), n_iter)
    return x.reshape(shape), hist


def modl_forward(aHy, S, m, weights, lam, T, n_cg):
    """MoDL with the soft operator: z = (D_W(x_1), x_2, ...), then the
    data-consistency solve.  Returns (x^T, states, zs)."""
    x = _c(aHy)
    states, zs = [x], []
    for _ in range(T):
        z = x.copy()
        z[:, 0] = cnn.denoise(x[:, 0], weights)
        x, _ = soft_cg_dc(aHy, z, S, m, lam, n_cg)
        zs.append(z)
        states.append(x)
    return x, states, zs


def coil_mse(x, S, ref):
    """Mean over all coil-image pixels of |sum_m S_{m,c} x_m - ref_c|^2."""
    d = coil_images(x, S) - _c(ref)
    return float(np.mean(np.abs(d) ** 2))


def coil_mse_grad(x, S, ref):
    """DF^H(1) gradient of ``coil_mse`` with respect to x: [B, M, H, W]."""
    d = coil_images(x, S) - _c(ref)
    return np.sum(np.conj(_c(S)) * (2.0 * d / d.size)[:, None], axis=2)


def modl_backward(g_out, states, zs, aHy, S, m, weights, lam, T, n_cg, bf16=False):
    """Reverse mode of ``modl_forward``.  Returns (grads, g_lambda [B], g_aHy).
    Each data-consistency block is differentiated by a second soft CG solve
    (v = S^{-1} g, g_aHy += v, g_z = lambda v, g_lambda += Re<v, z - x>); the
    denoiser's reverse pass acts on the first set only."""
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    g = _c(g_out)
    gW = [(np.zeros_like(np.asarray(Wt, dtype=np.float64)), np.zeros_like(np.asarray(b, dtype=np.float64)))
          for Wt, b in weights]
    g_lam = np.zeros(lam.shape)
    g_a = np.zeros_like(g)
    for t in range(T - 1, -1, -1):
        v, _ = soft_cg_dc(g, None, S, m, lam, n_cg)
        g_lam += np.sum(np.conj(v) * (zs[t] - states[t + 1]), axis=(1, 2, 3)).real
        g_a += v
        gz = lam[:, None, None, None] * v
        g = gz.copy()
        g0, lg = cnn.denoise_backward(states[t][:, 0], weights, gz[:, 0], bf16=bf16)
        g[:, 0] = g0
        gW = [(a[0] + b[0], a[1] + b[1]) for a, b in zip(gW, lg)]
    g_a += g
    return gW, g_lam, g_a
