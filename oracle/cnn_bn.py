"""The MoDL denoiser with batch normalisation (the MoDL subsection: L
convolution layers with F filters, batch normalisation and ReLU), in FP64.
Test infrastructure only: nothing in the product imports this module.

Each hidden layer l (the four 64-channel outputs) computes

    y_l = conv(a_{l-1}, W_l)                               (no bias)
    a_l = ReLU(gamma_l * (y_l - mu_l) / sqrt(var_l + eps) + beta_l)

with mu_l and var_l the mean and the biased variance of y_l over every pixel
of the batch (slices x rows x columns), per channel: the statistics of the
batch being processed (training-mode batch normalisation; it couples the
slices of a batch, as the paper notes for its MoDL).  The last layer is
conv + bias, linear, and the residual is added, as in ``oracle.cnn``.

Readings of what the paper leaves open: eps = 1e-5; the hidden convolutions
carry no bias (batch normalisation's beta takes its place, and a bias would
cancel in y - mu); every application of the shared denoiser in an unrolled
network normalises with its own batch's statistics.

bf16: as ``oracle.cnn`` -- the operands of every convolution (layer inputs,
weights, and in the reverse pass the gradient entering a convolution) are
rounded to bfloat16; statistics, normalisation, ReLU and their derivatives
stay float64.

Weights: ``weights`` as for ``oracle.cnn`` (the hidden biases are ignored);
``bn`` = [(gamma [64], beta [64]) for the four hidden layers].
"""
from __future__ import annotations

import numpy as np

from .cnn import _q, conv3x3, conv3x3_backward, from_channels, to_channels

EPS = 1e-5


def net_forward(x, weights, bn, keep=False, bf16=False):
    """N(x) for complex x [B,H,W]; with keep=True also the per-layer inputs,
    pre-normalisation outputs y, normalised values and inverse standard
    deviations."""
    a = _q(to_channels(x), bf16)
    acts, ys, yhats, istds = [], [], [], []
    L = len(weights)
    for l, (Wt, b) in enumerate(weights):
        acts.append(a)
        if l < L - 1:
            y = conv3x3(a, _q(Wt, bf16), np.zeros(Wt.shape[0]))
            mu = y.mean(axis=(0, 1, 2))
            var = ((y - mu) ** 2).mean(axis=(0, 1, 2))
            istd = 1.0 / np.sqrt(var + EPS)
            yhat = (y - mu) * istd
            g, be = (np.asarray(v, dtype=np.float64) for v in bn[l])
            a = _q(np.maximum(g * yhat + be, 0.0), bf16)
            ys.append(y)
            yhats.append(yhat)
            istds.append(istd)
        else:
            a = conv3x3(a, _q(Wt, bf16), b)
    out = from_channels(a)
    return (out, acts, ys, yhats, istds) if keep else out


def denoise(x, weights, bn, bf16=False):
    """D_W(x) = x + N(x)."""
    return np.asarray(x, dtype=np.complex128) + net_forward(x, weights, bn, bf16=bf16)


def denoise_backward(x, weights, bn, g, bf16=False):
    """Reverse mode of ``denoise`` at x with upstream gradient g (complex).
    Returns (g_x, [(gW, gb)] per layer (the hidden gb are zero), [(g_gamma,
    g_beta)] per hidden layer).  Through the normalisation with batch
    statistics, with z = gamma yhat + beta and g_z its gradient:
        g_beta = sum g_z,  g_gamma = sum g_z yhat,
        g_y = gamma istd (g_z - mean(g_z) - yhat mean(g_z yhat))
    (means over the batch's pixels, per channel)."""
    _, acts, ys, yhats, istds = net_forward(x, weights, bn, keep=True, bf16=bf16)
    L = len(weights)
    delta = to_channels(g)
    grads = [None] * L
    bn_grads = [None] * (L - 1)
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            gam, be = (np.asarray(v, dtype=np.float64) for v in bn[l])
            z = gam * yhats[l] + be
            gz = delta * (z > 0)
            g_beta = gz.sum(axis=(0, 1, 2))
            g_gamma = (gz * yhats[l]).sum(axis=(0, 1, 2))
            bn_grads[l] = (g_gamma, g_beta)
            delta = gam * istds[l] * (gz - gz.mean(axis=(0, 1, 2))
                                      - yhats[l] * (gz * yhats[l]).mean(axis=(0, 1, 2)))
        Wt = weights[l][0]
        ga, gW, _ = conv3x3_backward(acts[l], _q(Wt, bf16), _q(delta, bf16))
        # the last layer's bias gradient sums the unrounded gradient; the
        # hidden layers have no bias
        gb = delta.sum(axis=(0, 1, 2)) if l == L - 1 else np.zeros(Wt.shape[0])
        grads[l] = (gW, gb)
        delta = ga
    return from_channels(delta) + np.asarray(g, dtype=np.complex128), grads, bn_grads
