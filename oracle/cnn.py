"""Residual CNN denoiser D_W(x) = x + N(x) of the MoDL subsection, in FP64.

N is a stack of 3x3 convolution layers with bias; ReLU after every layer but
the last.  The complex image enters as two real channels (channel 0 = real
part, channel 1 = imaginary part) and leaves the same way.

Readings of points the paper leaves open (its MoDL uses batch normalisation
and F = 64 real filters; the configuration built here has no batch norm):

* convolution = cross-correlation with zero "same" padding,
  out[b,h,w,o] = bias[o] + sum_{dy,dx in {-1,0,1}} sum_i in[b,h+dy,w+dx,i] W[o,i,dy+1,dx+1];
* weights W [C_out, C_in, 3, 3], biases [C_out]; activations [B, H, W, C];
* the last layer is linear; the residual is added in the complex domain.

Gradients follow the DF^H(1) convention of the paper's complex-numbers
paragraph: for a complex quantity the returned gradient is dL/dRe + i dL/dIm.

Operand precision.  The configuration built here runs the convolutions with
bfloat16 operands and wide accumulation.  With ``bf16=True`` the oracle
computes exactly that definition: every operand of a convolution contraction
is rounded to bfloat16 (round to nearest even) --

* forward: the layer input (the complex image as two channels, or the
  previous layer's ReLU output) and the weights;
* reverse, input gradient: the gradient entering the layer (after the ReLU
  derivative) and the weights;
* reverse, weight gradient: the gradient entering the layer and the layer
  input --

while everything that is not a convolution operand stays float64: the sums,
biases, ReLU and its derivative (taken on the float64 pre-activation), the
bias gradients (sums of the unrounded gradient), the residual and the
network output.  The mode exists because the ReLU derivative is a decision on
a floating-point value: a bf16-operand network and the fp64 one disagree on
pre-activations within rounding of zero, so the decision has to be taken on
the same operands on both sides.  ``bf16=False`` (the default) is the plain
FP64 definition.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a):
    """Round to the nearest bfloat16 value (ties to even), via float32.
    Returns float64."""
    a32 = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a32.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(a, on):
    return bf16_round(a) if on else np.asarray(a, dtype=np.float64)


def _tap(ap, dy, dx, H, W):
    """The padded input shifted by tap (dy, dx), as a [pixels, channels] matrix."""
    return np.ascontiguousarray(ap[:, dy:dy + H, dx:dx + W, :]).reshape(-1, ap.shape[-1])


def conv3x3(a, Wt, bias):
    """Same-padded 3x3 cross-correlation. a [B,H,W,Ci], Wt [Co,Ci,3,3]."""
    a = np.asarray(a, dtype=np.float64)
    Wt = np.asarray(Wt, dtype=np.float64)
    B, H, W, _ = a.shape
    ap = np.pad(a, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((B * H * W, Wt.shape[0]))
    for dy in range(3):
        for dx in range(3):
            out += _tap(ap, dy, dx, H, W) @ np.ascontiguousarray(Wt[:, :, dy, dx].T)
    return out.reshape(B, H, W, -1) + np.asarray(bias, dtype=np.float64)


def conv3x3_backward(a, Wt, g):
    """Gradients of ``conv3x3`` w.r.t. its input, weights and bias given the
    output gradient g [B,H,W,Co]."""
    a = np.asarray(a, dtype=np.float64)
    Wt = np.asarray(Wt, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    B, H, W, _ = a.shape
    ap = np.pad(a, ((0, 0), (1, 1), (1, 1), (0, 0)))
    gp = np.pad(g, ((0, 0), (1, 1), (1, 1), (0, 0)))
    g2 = g.reshape(-1, g.shape[-1])
    ga = np.zeros((B * H * W, a.shape[-1]))
    gW = np.zeros_like(Wt)
    for dy in range(3):
        for dx in range(3):
            # out[p] uses in[p + d]  =>  g_in[q] += g[q - d] W_d
            ga += _tap(gp, 2 - dy, 2 - dx, H, W) @ np.ascontiguousarray(Wt[:, :, dy, dx])
            gW[:, :, dy, dx] = g2.T @ _tap(ap, dy, dx, H, W)
    gb = g.sum(axis=(0, 1, 2))
    return ga.reshape(a.shape), gW, gb


def to_channels(x):
    x = np.asarray(x, dtype=np.complex128)
    return np.stack([x.real, x.imag], axis=-1)


def from_channels(a):
    return a[..., 0] + 1j * a[..., 1]


def net_forward(x, weights, keep=False, bf16=False):
    """N(x) for complex x [B,H,W]; weights = [(W, b), ...].
    With keep=True also returns the per-layer inputs and pre-activations.
    bf16: round the layer inputs and the weights to bfloat16 (see module)."""
    a = _q(to_channels(x), bf16)
    acts, pres = [], []
    L = len(weights)
    for l, (Wt, b) in enumerate(weights):
        acts.append(a)
        pre = conv3x3(a, _q(Wt, bf16), b)
        pres.append(pre)
        a = _q(np.maximum(pre, 0.0), bf16) if l < L - 1 else pre
    out = from_channels(a)
    return (out, acts, pres) if keep else out


def denoise(x, weights, bf16=False):
    """D_W(x) = x + N(x)."""
    return np.asarray(x, dtype=np.complex128) + net_forward(x, weights, bf16=bf16)


def denoise_backward(x, weights, g, bf16=False, keep=False):
    """Reverse mode of D_W at x with upstream gradient g (complex [B,H,W]).
    Returns (g_x complex, [(gW, gb), ...]), and with keep=True also the
    gradients with respect to each layer's pre-activation (the bias
    gradients are their sums over pixels).  With bf16=True the operands of
    the reverse convolutions are rounded to bfloat16 as described in the
    module docstring; bias gradients sum the unrounded gradient."""
    _, acts, pres = net_forward(x, weights, keep=True, bf16=bf16)
    L = len(weights)
    delta = to_channels(g)
    grads, deltas = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            delta = delta * (pres[l] > 0)
        deltas[l] = delta
        gin, gW, _ = conv3x3_backward(acts[l], _q(weights[l][0], bf16), _q(delta, bf16))
        grads[l] = (gW, delta.sum(axis=(0, 1, 2)))
        delta = gin
    gx = np.asarray(g, dtype=np.complex128) + from_channels(delta)
    return (gx, grads, deltas) if keep else (gx, grads)


def n_params(channels, k=3):
    """Weights plus biases of a plain conv stack."""
    return sum(channels[i] * channels[i + 1] * k * k + channels[i + 1]
               for i in range(len(channels) - 1))
