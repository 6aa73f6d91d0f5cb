"""Non-Cartesian SENSE through the Toeplitz form of its normal operator
(Extensions to the SENSE-Model subsection), in FP64.  Test infrastructure
only: nothing in the product imports this module.

The sampling is a list of M k-space points k_j = (ky_j, kx_j) in cycles per
field of view; the Cartesian grid point of row index l of an H-row k-space
is ky = l - H/2.  The forward operator evaluates the Fourier transform of
each coil image at those points (a non-uniform DFT, computed here by its
definition, not by gridding):

    y_{c,j} = (HW)^{-1/2} sum_{r,s} S_c[r,s] x[r,s]
              exp(-2 pi i (ky_j (r - H/2) / H + kx_j (s - W/2) / W)),

and A^H is its exact adjoint.  The scale makes a trajectory that covers the
Cartesian grid once reproduce the centred unitary DFT of ``oracle.sense``.

Toeplitz form (the PSF convolution the paper uses for F^H P^H P F): for one
coil image u, (F^H P^H P F u)[n] = sum_m u[m] h[n - m], a convolution with
the point spread function

    h[dy, dx] = (HW)^{-1} sum_j exp(+2 pi i (ky_j dy / H + kx_j dx / W)),
    |dy| < H, |dx| < W.

A linear convolution over offsets below (H, W) is a cyclic one on a grid of
2H x 2W: u is zero-padded into the top-left H x W corner, h is laid out
cyclically (h[dy, dx] at (dy mod 2H, dx mod 2W), zero on row H and column
W), and

    F^H P^H P F u = crop( IDFT_2( psf * DFT_2( pad(u) ) ) ),  psf = DFT_2(h),

with DFT_2 the unnormalised 2H x 2W DFT and IDFT_2 its inverse.  h is
Hermitian (h[-d] = conj h[d]), so psf is real.

Readings of what the paper leaves open:

* no density compensation inside the normal operator (weights 1): A^H A is
  the exact Gram operator of the sampling;
* the non-Cartesian networks start from the SENSE reconstruction
  x^0 = (A^H A + lambda I)^{-1} A^H y by the same CG recipe (its lambda and
  iteration count those of the data-consistency blocks);
* MoDL otherwise as ``oracle.modl`` with the normal operator replaced.

Shapes: x [B, H, W], S [B, C, H, W], traj [B, M, 2] (ky, kx), y [B, C, M],
psf [B, 2H, 2W] (real).
"""
from __future__ import annotations

import numpy as np

from . import cg as ocg
from . import cnn


def _c(a):
    return np.asarray(a).astype(np.complex128)


def _phase(traj, H, W):
    """[M, H, W] array exp(-2 pi i (ky (r - H/2)/H + kx (s - W/2)/W))."""
    t = np.asarray(traj, dtype=np.float64)
    r = np.arange(H) - H // 2
    s = np.arange(W) - W // 2
    ey = np.exp(-2j * np.pi * np.outer(t[:, 0], r) / H)  # [M, H]
    ex = np.exp(-2j * np.pi * np.outer(t[:, 1], s) / W)  # [M, W]
    return ey[:, :, None] * ex[:, None, :]


def nudft_fwd(x, S, traj):
    """y [B, C, M] = A x (no noise)."""
    x, S = _c(x), _c(S)
    B, C, H, W = S.shape
    y = []
    for b in range(B):
        E = _phase(traj[b], H, W).reshape(-1, H * W)  # [M, HW]
        u = (S[b] * x[b][None]).reshape(C, H * W)
        y.append(u @ E.T / np.sqrt(H * W))
    return np.stack(y)


def nudft_adj(y, S, traj):
    """x [B, H, W] = A^H y = sum_c conj(S_c) F_nu^H y_c."""
    y, S = _c(y), _c(S)
    B, C, H, W = S.shape
    out = []
    for b in range(B):
        E = _phase(traj[b], H, W).reshape(-1, H * W)
        u = (y[b] @ np.conj(E)).reshape(C, H, W) / np.sqrt(H * W)
        out.append(np.sum(np.conj(S[b]) * u, axis=0))
    return np.stack(out)


def normal_direct(x, S, traj, lam=0.0):
    """(A^H A + lambda I) x by the definition (forward then adjoint)."""
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64).reshape(-1), (np.shape(x)[0],))
    return nudft_adj(nudft_fwd(x, S, traj), S, traj) + lam[:, None, None] * _c(x)


def psf_kernel(traj, H, W):
    """h on the cyclic 2H x 2W layout (complex), one slice."""
    t = np.asarray(traj, dtype=np.float64)
    dy = np.arange(-(H - 1), H)
    dx = np.arange(-(W - 1), W)
    ey = np.exp(2j * np.pi * np.outer(t[:, 0], dy) / H)  # [M, 2H-1]
    ex = np.exp(2j * np.pi * np.outer(t[:, 1], dx) / W)  # [M, 2W-1]
    h = ey.T @ ex / (H * W)  # [2H-1, 2W-1], sum over j
    c = np.zeros((2 * H, 2 * W), dtype=np.complex128)
    c[np.ix_(dy % (2 * H), dx % (2 * W))] = h
    return c


def psf_spectrum(traj, H, W):
    """psf [B, 2H, 2W]: the unnormalised 2-D DFT of the cyclic kernel; real
    up to rounding (returned complex so that callers can check it)."""
    return np.stack([np.fft.fft2(psf_kernel(t, H, W)) for t in traj])


def psf(traj, H, W):
    """Real psf [B, 2H, 2W]."""
    return psf_spectrum(traj, H, W).real


def toeplitz_1(u, P):
    """crop(IDFT_2(P * DFT_2(pad u))) for images u [..., H, W], P [2H, 2W]."""
    u = _c(u)
    H, W = u.shape[-2:]
    pad = np.zeros(u.shape[:-2] + (2 * H, 2 * W), dtype=np.complex128)
    pad[..., :H, :W] = u
    return np.fft.ifft2(P * np.fft.fft2(pad))[..., :H, :W]


def normal(x, S, P, lam=0.0):
    """(A^H A + lambda I) x through the PSF: sum_c conj(S_c) T(S_c x) + lambda x."""
    x, S = _c(x), _c(S)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64).reshape(-1), (x.shape[0],))
    out = np.stack([np.sum(np.conj(S[b]) * toeplitz_1(S[b] * x[b][None], P[b]), axis=0)
                    for b in range(x.shape[0])])
    return out + lam[:, None, None] * x


def cg_dc(aHy, z, S, P, lam, n_iter):
    """x = (A^H A + lambda I)^{-1} (aHy + lambda z) by ``oracle.cg.cg``."""
    aHy = _c(aHy)
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64).reshape(-1), (aHy.shape[0],))
    rhs = aHy if z is None else aHy + lam[:, None, None] * _c(z)
    return ocg.cg(lambda v: normal(v, S, P, lam), rhs, n_iter)


def sense_init(aHy, S, P, lam, n_iter):
    """x^0 = (A^H A + lambda I)^{-1} A^H y: the SENSE reconstruction the
    non-Cartesian networks start from."""
    return cg_dc(aHy, None, S, P, lam, n_iter)[0]


def modl_forward(x0, aHy, S, P, weights, lam, T, n_cg, bf16=False):
    """MoDL from x^0: x^{t+1} = (A^H A + lambda I)^{-1}(aHy + lambda D(x^t)).
    Returns (x^T, states [x^0..x^T], zs)."""
    x = _c(x0)
    states, zs = [x], []
    for _ in range(T):
        z = cnn.denoise(x, weights, bf16=bf16)
        x, _ = cg_dc(aHy, z, S, P, lam, n_cg)
        zs.append(z)
        states.append(x)
    return x, states, zs


def modl_backward(g_out, states, zs, aHy, S, P, weights, lam, T, n_cg, bf16=False):
    """Reverse mode of ``modl_forward`` (as ``oracle.modl.backward``, the
    data-consistency blocks through the PSF form): each block's adjoint is
    v = (A^H A + lambda I)^{-1} g (self-adjoint), g_z = lambda v,
    g_lambda = Re<v, z - x>.  Returns (grads [(gW, gb)], g_lambda [B],
    g_aHy, g_x0)."""
    lam = np.broadcast_to(np.asarray(lam, dtype=np.float64).reshape(-1), (np.shape(aHy)[0],))
    g = _c(g_out)
    gW = [(np.zeros_like(np.asarray(W, dtype=np.float64)),
           np.zeros_like(np.asarray(b, dtype=np.float64))) for W, b in weights]
    g_lam = np.zeros(lam.shape)
    g_a = np.zeros_like(g)
    for t in range(T - 1, -1, -1):
        v, _ = ocg.cg(lambda u: normal(u, S, P, lam), g, n_cg)
        g_lam += np.sum(np.conj(v) * (_c(zs[t]) - _c(states[t + 1])), axis=(-2, -1)).real
        g_a += v
        g, lg = cnn.denoise_backward(states[t], weights, lam[:, None, None] * v, bf16=bf16)
        gW = [(a[0] + b[0], a[1] + b[1]) for a, b in zip(gW, lg)]
    return gW, g_lam, g_a, g


def nudft_adj_pixels(y, S, traj, pixels):
    """A^H y at the listed pixels only ([(b, r, s), ...]): the definition
    evaluated one pixel at a time (for spot checks of large images)."""
    y, S = _c(y), _c(S)
    _, C, H, W = S.shape
    out = []
    for b, r, s in pixels:
        t = np.asarray(traj[b], dtype=np.float64)
        e = np.exp(2j * np.pi * (t[:, 0] * (r - H // 2) / H + t[:, 1] * (s - W // 2) / W))
        u = y[b] @ e / np.sqrt(H * W)  # [C]
        out.append(np.sum(np.conj(S[b, :, r, s]) * u))
    return np.array(out)


def nudft_fwd_samples(x, S, traj, samples):
    """A x at the listed samples only ([(b, j), ...]) -> [len, C]: the
    definition evaluated one sample at a time (for spot checks)."""
    x, S = _c(x), _c(S)
    _, C, H, W = S.shape
    r = np.arange(H) - H // 2
    s = np.arange(W) - W // 2
    out = []
    for b, j in samples:
        ky, kx = np.asarray(traj[b][j], dtype=np.float64)
        e = np.exp(-2j * np.pi * (ky * r[:, None] / H + kx * s[None, :] / W))
        out.append(np.sum(S[b] * x[b][None] * e[None], axis=(1, 2)) / np.sqrt(H * W))
    return np.array(out)
