"""SENSE operator A = P F C in FP64 (Methods, Applications and Implemented
Networks: the inverse problem eq. inverse_problem and the SENSE operator
composed of coil multiplication C, Fourier transform F and sampling
projection P).

Readings of points the paper leaves open:

* F is the centered, unitary 2-D DFT (DC at index N//2, forward kernel
  exp(-2 pi i k n / N), scale 1/sqrt(N) per axis).  Unitarity is what makes
  A^H A the identity at full sampling when sum_c |S_c|^2 = 1.
* P is the projection onto sampled phase-encode lines; a mask value
  m[h] in {0, 1} per row (h along H), constant along the readout W.  Then
  P^H P = diag(m) and the forward output keeps zeros on unsampled rows.
* Shapes: x [B, H, W], S [B, C, H, W], m [B, H], y [B, C, H, W].
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft


def _c128(a):
    return np.asarray(a).astype(np.complex128)


def fft1c(x, axis):
    """Centered unitary 1-D DFT along ``axis``."""
    return sfft.fftshift(
        sfft.fft(sfft.ifftshift(x, axes=axis), axis=axis, norm="ortho"), axes=axis)


def ifft1c(x, axis):
    """Inverse (= adjoint) of ``fft1c``."""
    return sfft.fftshift(
        sfft.ifft(sfft.ifftshift(x, axes=axis), axis=axis, norm="ortho"), axes=axis)


def fft2c(x):
    """Centered unitary 2-D DFT over the last two axes (H, W)."""
    return fft1c(fft1c(x, -1), -2)


def ifft2c(x):
    return ifft1c(ifft1c(x, -1), -2)


def _rowmask(m):
    m = np.asarray(m, dtype=np.float64)
    return m[:, None, :, None]  # [B, 1, H, 1]


def sense_fwd(x, S, m):
    """y_c = P F (S_c x): coil images, 2-D centered FFT, row sampling."""
    x, S = _c128(x), _c128(S)
    return _rowmask(m) * fft2c(S * x[:, None])


def sense_adj(y, S, m):
    """x = sum_c conj(S_c) F^H P^H y_c."""
    y, S = _c128(y), _c128(S)
    return np.sum(np.conj(S) * ifft2c(_rowmask(m) * y), axis=1)


def sense_normal(x, S, m, lam):
    """(A^H A + lambda I) x with one lambda per slice."""
    lam = np.asarray(lam, dtype=np.float64).reshape(-1, 1, 1)
    return sense_adj(sense_fwd(x, S, m), S, m) + lam * _c128(x)


def measure(x, S, m, noise):
    """Training-data forward model of the Results section: coil images,
    Fourier transform, additive complex Gaussian noise, subsampling.
    y = P (F (S x) + n)."""
    return _rowmask(m) * (fft2c(_c128(S) * _c128(x)[:, None]) + _c128(noise))


def sense_normal_1d(x, S, m, lam):
    """The same normal operator written through 1-D transforms along H only.

    Because the mask is constant along W and the W-transform is unitary and
    acts on a different axis than the mask, F^H P^H P F = F_H^H diag(m) F_H
    (the W transforms cancel).  Used only to pin that identity, which the GPU
    kernels rely on, against the literal 2-D form.
    """
    x, S = _c128(x), _c128(S)
    lam = np.asarray(lam, dtype=np.float64).reshape(-1, 1, 1)
    v = fft1c(S * x[:, None], -2)
    v = _rowmask(m) * v
    return np.sum(np.conj(S) * ifft1c(v, -2), axis=1) + lam * x
