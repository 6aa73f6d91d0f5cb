"""Variational-network stage (Variational Network subsection, eq. update_vn)
in FP64:

    x' = x - sum_i K_i^T Phi'_i(K_i x) - lambda (A^H A x - A^H y)

K_i is a convolution of the complex image with a complex N_k x N_k filter
k_i whose imaginary part is discarded (as the paper states, for consistency
with the original VarNet): s_i = Re(k_i * x).  Phi'_i is a trainable
activation, a weighted sum of N_w Gaussian radial basis functions.

Readings of points the paper leaves open:

* "*" is cross-correlation with zero "same" padding:
  s_i[p] = sum_d Re k_i[d] Re x[p+d] - Im k_i[d] Im x[p+d], d in [-r, r]^2;
  K_i^T is its exact adjoint for the real inner product Re<.,.>.
* RBF knots mu_j = -1 + 2 j / (N_w - 1) on [-1, 1]; width sigma = the knot
  spacing 2 / (N_w - 1);  Phi'_i(s) = sum_j w_ij exp(-(s - mu_j)^2 / (2 sigma^2)).
* Parameters per stage: N_k complex filters (2 N_k r^2 reals), N_k x N_w RBF
  weights, one step size lambda -- 65,530 real parameters for the defaults
  T = 10, N_k = 24, 11 x 11, N_w = 31 quoted in the paper.
* Gradients use the DF^H(1) convention (dL/dRe + i dL/dIm).
"""
from __future__ import annotations

import numpy as np

from . import sense


def n_params(T=10, n_filters=24, ksize=11, n_rbf=31):
    return T * (n_filters * ksize * ksize * 2 + n_filters * n_rbf + 1)


def knots(n_rbf):
    mu = -1.0 + 2.0 * np.arange(n_rbf) / (n_rbf - 1)
    return mu, 2.0 / (n_rbf - 1)


def filt(x, k):
    """s[b,i,h,w] = Re(k_i * x) for complex x [B,H,W], k [Nk,ks,ks]."""
    x = np.asarray(x, dtype=np.complex128)
    k = np.asarray(k, dtype=np.complex128)
    B, H, W = x.shape
    Nk, ks, _ = k.shape
    r = ks // 2
    xp = np.pad(x, ((0, 0), (r, r), (r, r)))
    s = np.zeros((B, Nk, H, W))
    for dy in range(ks):
        for dx in range(ks):
            sh = xp[:, dy:dy + H, dx:dx + W]
            s += (k[None, :, dy, dx, None, None].real * sh.real[:, None]
                  - k[None, :, dy, dx, None, None].imag * sh.imag[:, None])
    return s


def filt_adj(u, k):
    """K^T u: complex [B,H,W] from real u [B,Nk,H,W] (adjoint of ``filt``)."""
    u = np.asarray(u, dtype=np.float64)
    k = np.asarray(k, dtype=np.complex128)
    B, Nk, H, W = u.shape
    ks = k.shape[-1]
    r = ks // 2
    up = np.pad(u, ((0, 0), (0, 0), (r, r), (r, r)))
    out = np.zeros((B, H, W), dtype=np.complex128)
    for dy in range(ks):
        for dx in range(ks):
            # s[p] used x[p+d]  =>  adjoint gathers u[q-d]
            sh = up[:, :, 2 * r - dy:2 * r - dy + H, 2 * r - dx:2 * r - dx + W]
            kr = k[:, dy, dx].real[None, :, None, None]
            ki = k[:, dy, dx].imag[None, :, None, None]
            out += np.sum(kr * sh, axis=1) - 1j * np.sum(ki * sh, axis=1)
    return out


def rbf(s, w):
    """Phi'(s) and Phi''(s) for s [B,Nk,H,W], w [Nk,Nw]."""
    w = np.asarray(w, dtype=np.float64)
    mu, sig = knots(w.shape[-1])
    d = s[..., None] - mu  # [B,Nk,H,W,Nw]
    e = np.exp(-d * d / (2 * sig * sig))
    wb = w[None, :, None, None, :]
    return np.sum(wb * e, axis=-1), np.sum(wb * e * (-d / (sig * sig)), axis=-1), e


def stage(x, aHy, S, m, k, w, lam):
    x = np.asarray(x, dtype=np.complex128)
    s = filt(x, k)
    phi1, _, _ = rbf(s, w)
    lam_b = np.full(x.shape[0], float(lam))
    dc = sense.sense_normal(x, S, m, np.zeros_like(lam_b)) - np.asarray(aHy, np.complex128)
    return x - filt_adj(phi1, k) - float(lam) * dc


def stage_backward(g, x, aHy, S, m, k, w, lam):
    """Returns (g_x, g_k complex [Nk,ks,ks], g_w [Nk,Nw], g_lam scalar)."""
    g = np.asarray(g, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128)
    k = np.asarray(k, dtype=np.complex128)
    B = x.shape[0]
    zero = np.zeros(B)
    s = filt(x, k)
    phi1, phi2, e = rbf(s, w)
    Kg = filt(g, k)
    ee = phi2 * Kg
    AHAx = sense.sense_normal(x, S, m, zero)
    g_x = g - filt_adj(ee, k) - float(lam) * sense.sense_normal(g, S, m, zero)
    g_lam = -float(np.sum(np.real(np.conj(g) * (AHAx - np.asarray(aHy, np.complex128)))))
    g_w = -np.einsum("bihw,bihwj->ij", Kg, e)
    ks = k.shape[-1]
    r = ks // 2
    H, W = x.shape[1:]
    gp = np.pad(g, ((0, 0), (r, r), (r, r)))
    xp = np.pad(x, ((0, 0), (r, r), (r, r)))
    g_k = np.zeros(k.shape, dtype=np.complex128)
    for dy in range(ks):
        for dx in range(ks):
            gs = gp[:, dy:dy + H, dx:dx + W]
            xs = xp[:, dy:dy + H, dx:dx + W]
            dkr = -(np.einsum("bihw,bhw->i", phi1, gs.real)
                    + np.einsum("bihw,bhw->i", ee, xs.real))
            dki = (np.einsum("bihw,bhw->i", phi1, gs.imag)
                   + np.einsum("bihw,bhw->i", ee, xs.imag))
            g_k[:, dy, dx] = dkr + 1j * dki
    return g_x, g_k, g_w, g_lam


def forward(aHy, S, m, params, T=None):
    """x^0 = A^H y, then T stages.  Returns (x^T, states)."""
    T = params["k"].shape[0] if T is None else T
    x = np.asarray(aHy, dtype=np.complex128)
    states = [x]
    for t in range(T):
        x = stage(x, aHy, S, m, params["k"][t], params["w"][t], params["lam"][t])
        states.append(x)
    return x, states


def backward(g_out, states, aHy, S, m, params, T=None):
    T = params["k"].shape[0] if T is None else T
    g = np.asarray(g_out, dtype=np.complex128)
    gk = np.zeros(params["k"][:T].shape, dtype=np.complex128)
    gw = np.zeros(params["w"][:T].shape)
    gl = np.zeros(T)
    g_a = np.zeros_like(g)
    for t in range(T - 1, -1, -1):
        lam = params["lam"][t]
        g_a += float(lam) * g  # x' contains + lambda A^H y
        g, gk[t], gw[t], gl[t] = stage_backward(
            g, states[t], aHy, S, m, params["k"][t], params["w"][t], lam)
    g_a += g
    return gk, gw, gl, g_a
