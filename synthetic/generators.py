"""Seeded generators for phantoms, coil maps, phase-encode masks, noise, weights.

Recipe (stand-in for the knee and brain datasets of the paper's Results
section, which are not available here):

* Phantom: on normalised coordinates u (readout, along W) and v (phase
  encode, along H), both in [-1, 1), a sum of K ~ U{8..14} filled ellipses with
  centre ~ U(-0.6, 0.6)^2, semi-axes ~ U(0.05, 0.45), angle ~ U(0, pi) and
  amplitude ~ U(0.1, 1); the magnitude is divided by its maximum so it lies in
  [0, 1].  A smooth quadratic phase c0 + c1 u + c2 v + c3 u^2 + c4 v^2 + c5 u v
  with c ~ U(-pi/4, pi/4) is applied.
* Coils: C Gaussian profiles (width 0.7) centred on a circle of radius 1.3 at
  angle 2 pi c / C + U(-0.1, 0.1), with a linear phase ramp, normalised so that
  sum_c |S_c|^2 = 1 at every pixel.
* Masks: phase-encode lines (rows).  floor(H / R) lines in total including a
  fully sampled centre block; the rest drawn without replacement either
  uniformly or with variable density p ~ (1 - |k - H/2| / (H/2))^2 + 1e-3; or
  the regular pattern (every R-th line plus a centre block).
* Noise: sigma * (N(0,1) + i N(0,1)) per k-space sample, sigma = 1e-3 (the
  paper's training-data recipe, Results section).
* Non-Cartesian: radial spokes through the centre with a random rotation
  per slice (``radial_trajectory``), the same phantoms and coil maps.

Everything is drawn in float64 with ``numpy.random.default_rng(seed)`` and
rounded once to complex64 / float32.
"""
from __future__ import annotations

import math

import numpy as np

# Seed conventions: config k test inputs use 1000*k + slice index; training
# phantoms, held-out evaluation phantoms and weights have their own ranges.
SEEDS = {
    "train_base": 100000,
    "train_count": 2000,
    "eval_base": 200000,
    "eval_count": 64,
    "weights": 7,
}


def _grid(H: int, W: int):
    v = -1.0 + 2.0 * np.arange(H, dtype=np.float64) / H
    u = -1.0 + 2.0 * np.arange(W, dtype=np.float64) / W
    return np.meshgrid(v, u, indexing="ij")  # (V, U), each [H, W]


def phantom(seed: int, H: int, W: int) -> np.ndarray:
    """Random-ellipse complex phantom, magnitude in [0, 1]; complex64 [H, W]."""
    rng = np.random.default_rng(seed)
    V, U = _grid(H, W)
    K = int(rng.integers(8, 15))
    mag = np.zeros((H, W), dtype=np.float64)
    for _ in range(K):
        cu, cv = rng.uniform(-0.6, 0.6, size=2)
        a, b = rng.uniform(0.05, 0.45, size=2)
        th = rng.uniform(0.0, math.pi)
        amp = rng.uniform(0.1, 1.0)
        du, dv = U - cu, V - cv
        ru = du * math.cos(th) + dv * math.sin(th)
        rv = -du * math.sin(th) + dv * math.cos(th)
        mag += amp * (((ru / a) ** 2 + (rv / b) ** 2) <= 1.0)
    mx = mag.max()
    if mx > 0:
        mag /= mx
    c = rng.uniform(-math.pi / 4, math.pi / 4, size=6)
    phi = c[0] + c[1] * U + c[2] * V + c[3] * U * U + c[4] * V * V + c[5] * U * V
    return (mag * np.exp(1j * phi)).astype(np.complex64)


def coil_maps(seed: int, C: int, H: int, W: int) -> np.ndarray:
    """C Gaussian coil profiles with sum_c |S_c|^2 = 1; complex64 [C, H, W]."""
    rng = np.random.default_rng(seed)
    V, U = _grid(H, W)
    S = np.empty((C, H, W), dtype=np.complex128)
    for c in range(C):
        th = 2 * math.pi * c / C + rng.uniform(-0.1, 0.1)
        cu, cv = 1.3 * math.cos(th), 1.3 * math.sin(th)
        prof = np.exp(-((U - cu) ** 2 + (V - cv) ** 2) / (2 * 0.7 ** 2))
        ph = 2 * math.pi * c / C + 0.3 * (U * math.cos(th) + V * math.sin(th))
        S[c] = prof * np.exp(1j * ph)
    S /= np.sqrt(np.sum(np.abs(S) ** 2, axis=0, keepdims=True))
    return S.astype(np.complex64)


def pe_mask(seed: int, H: int, R: int, n_center: int, kind: str = "vd") -> np.ndarray:
    """Phase-encode line mask, float32 [H] with values in {0, 1}.

    kind = "uniform": centre block plus uniform random lines;
    kind = "vd": centre block plus variable-density random lines;
    kind = "regular": every R-th line plus the centre block.
    """
    m = np.zeros(H, dtype=np.float32)
    c0 = H // 2 - n_center // 2
    m[c0:c0 + n_center] = 1.0
    if kind == "regular":
        m[::R] = 1.0
        return m
    rng = np.random.default_rng(seed)
    n_tot = H // R
    n_rest = max(0, n_tot - int(m.sum()))
    cand = np.flatnonzero(m == 0)
    if kind == "uniform":
        p = np.ones(cand.size, dtype=np.float64)
    elif kind == "vd":
        p = (1.0 - np.abs(cand - H / 2) / (H / 2)) ** 2 + 1e-3
    else:
        raise ValueError(kind)
    p = p / p.sum()
    pick = rng.choice(cand, size=min(n_rest, cand.size), replace=False, p=p)
    m[pick] = 1.0
    return m


def kspace_noise(seed: int, C: int, H: int, W: int, sigma: float = 1e-3) -> np.ndarray:
    """Complex Gaussian noise, sigma per real component; complex64 [C, H, W]."""
    rng = np.random.default_rng(seed)
    n = rng.standard_normal((C, H, W, 2))
    return (sigma * (n[..., 0] + 1j * n[..., 1])).astype(np.complex64)


CNN_CHANNELS = (2, 64, 64, 64, 64, 2)


def cnn_weights(seed: int = 7, channels=CNN_CHANNELS, last_scale: float = 1.0):
    """He-normal 3x3 conv weights N(0, 2/(9 C_in)), zero biases.

    Returns a list of (W [C_out, C_in, 3, 3] float32, b [C_out] float32).
    ``last_scale`` multiplies the last layer (1.0 = plain He init).
    """
    rng = np.random.default_rng(seed)
    out = []
    L = len(channels) - 1
    for l in range(L):
        ci, co = channels[l], channels[l + 1]
        std = math.sqrt(2.0 / (9 * ci))
        Wt = rng.standard_normal((co, ci, 3, 3)) * std
        if l == L - 1:
            Wt = Wt * last_scale
        out.append((Wt.astype(np.float32), np.zeros(co, dtype=np.float32)))
    return out


def vn_params(seed: int, n_stages: int = 10, n_filters: int = 24, ksize: int = 11,
              n_rbf: int = 31, lam0: float = 0.1):
    """Initial variational-network parameters for ``n_stages`` stages.

    Filters: complex, real and imaginary parts N(0, 0.01) (std 0.1) with the
    per-filter mean removed.  RBF weights w_ij = 0.1 * mu_j / sqrt(2 pi), which
    makes the activation close to 0.1 * s on [-1, 1] when the Gaussian width
    equals the knot spacing.  Step sizes lambda_t = lam0.
    Returns dict of float32 / complex64 arrays:
      k [T, N_k, ks, ks] complex64, w [T, N_k, N_w] float32, lam [T] float32.
    """
    rng = np.random.default_rng(seed)
    k = (rng.standard_normal((n_stages, n_filters, ksize, ksize))
         + 1j * rng.standard_normal((n_stages, n_filters, ksize, ksize))) * 0.1
    k -= k.mean(axis=(2, 3), keepdims=True)
    mu = -1.0 + 2.0 * np.arange(n_rbf) / (n_rbf - 1)
    w = np.broadcast_to(0.1 * mu / math.sqrt(2 * math.pi), (n_stages, n_filters, n_rbf))
    return {
        "k": k.astype(np.complex64),
        "w": np.ascontiguousarray(w).astype(np.float32),
        "lam": np.full(n_stages, lam0, dtype=np.float32),
    }


def slice_inputs(seed: int, H: int, W: int, C: int, R: int, n_center: int,
                 mask_kind: str = "vd", sigma: float = 1e-3):
    """One slice: phantom x [H,W], coils S [C,H,W], mask m [H], noise n [C,H,W].

    The four draws use seeds derived from ``seed`` so that each is reproducible
    on its own.
    """
    return {
        "x": phantom(seed, H, W),
        "S": coil_maps(seed + 7919, C, H, W),
        "mask": pe_mask(seed + 15485863, H, R, n_center, mask_kind),
        "noise": kspace_noise(seed + 32452843, C, H, W, sigma),
    }


def soft_slice_inputs(seed: int, H: int, W: int, C: int, R: int, n_center: int,
                      mask_kind: str = "vd", sigma: float = 1e-3):
    """One slice whose object is larger than the field of view along H (the
    reduced-FOV setting of the paper's soft-SENSE experiment), laid out for
    two sets of coil maps: phantom and coil maps are drawn on a 2H x W grid;
    the field of view is its central H rows and the other H rows are the
    ones that alias into it.  Returns x [2, H, W] (set 0: the field of view,
    set 1: the aliasing rows, row i of set 1 being extended row
    (i + 3H/2) mod 2H), S [2, C, H, W] arranged the same way, mask [H] and
    noise [C, H, W] for the H-row k-space.  Only draws and index
    rearrangements (rolls and slices) happen here."""
    xe = phantom(seed, 2 * H, W)
    Se = coil_maps(seed + 7919, C, 2 * H, W)
    xr = np.roll(xe, -(H // 2), axis=0)
    Sr = np.roll(Se, -(H // 2), axis=1)
    return {
        "x": np.ascontiguousarray(np.stack([xr[:H], xr[H:]])),
        "S": np.ascontiguousarray(np.stack([Sr[:, :H], Sr[:, H:]])),
        "mask": pe_mask(seed + 15485863, H, R, n_center, mask_kind),
        "noise": kspace_noise(seed + 32452843, C, H, W, sigma),
        "x_ext": xe,
        "S_ext": Se,
    }


def soft_batch_inputs(seeds, H: int, W: int, C: int, R: int, n_center: int,
                      mask_kind: str = "vd", sigma: float = 1e-3):
    """Stack ``soft_slice_inputs``: x [B,2,H,W], S [B,2,C,H,W], mask [B,H],
    noise [B,C,H,W] (and the extended x_ext [B,2H,W], S_ext [B,C,2H,W])."""
    sl = [soft_slice_inputs(s, H, W, C, R, n_center, mask_kind, sigma) for s in seeds]
    return {k: np.stack([d[k] for d in sl]) for k in sl[0]}


def batch_inputs(seeds, H: int, W: int, C: int, R: int, n_center: int,
                 mask_kind: str = "vd", sigma: float = 1e-3):
    """Stack ``slice_inputs`` over ``seeds``: x [B,H,W], S [B,C,H,W], mask [B,H],
    noise [B,C,H,W]."""
    sl = [slice_inputs(s, H, W, C, R, n_center, mask_kind, sigma) for s in seeds]
    return {k: np.stack([d[k] for d in sl]) for k in sl[0]}


def radial_trajectory(seed: int, H: int, W: int, n_spokes: int, n_read: int) -> np.ndarray:
    """Radial sampling (the paper's non-Cartesian experiment uses 44 spokes):
    n_spokes lines through the k-space centre at angles
    theta_s = theta_0 + pi s / n_spokes (theta_0 ~ U(0, pi / n_spokes)), each
    with n_read equispaced samples t_i = (i - n_read / 2) / n_read, i <
    n_read, of the extent; returns traj [n_spokes * n_read, 2] float32 of
    (ky, kx) = (t_i H sin theta_s, t_i W cos theta_s) in cycles per field
    of view (so the samples span [-H/2, H/2) x [-W/2, W/2))."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(0.0, math.pi / n_spokes) + math.pi * np.arange(n_spokes) / n_spokes
    t = (np.arange(n_read) - n_read / 2) / n_read
    ky = np.outer(np.sin(th), t) * H
    kx = np.outer(np.cos(th), t) * W
    return np.stack([ky.ravel(), kx.ravel()], axis=1).astype(np.float32)


def noncart_slice_inputs(seed: int, H: int, W: int, C: int, n_spokes: int, n_read: int,
                         sigma: float = 1e-3):
    """One non-Cartesian slice: phantom x [H,W], coils S [C,H,W], radial
    trajectory traj [M,2] (M = n_spokes n_read) and noise [C,M]."""
    M = n_spokes * n_read
    rng = np.random.default_rng(seed + 32452843)
    n = sigma * (rng.standard_normal((C, M)) + 1j * rng.standard_normal((C, M)))
    return {
        "x": phantom(seed, H, W),
        "S": coil_maps(seed + 7919, C, H, W),
        "traj": radial_trajectory(seed + 15485863, H, W, n_spokes, n_read),
        "noise": n.astype(np.complex64),
    }


def noncart_batch_inputs(seeds, H: int, W: int, C: int, n_spokes: int, n_read: int, sigma: float = 1e-3):
    """Stack ``noncart_slice_inputs``: x [B,H,W], S [B,C,H,W], traj [B,M,2],
    noise [B,C,M]."""
    sl = [noncart_slice_inputs(s, H, W, C, n_spokes, n_read, sigma) for s in seeds]
    return {k: np.stack([d[k] for d in sl]) for k in sl[0]}


# Matrix sizes of the uneven-batch workload (H x W), drawn per slice.
UNEVEN_SHAPES = ((192, 192), (256, 256), (320, 320), (384, 320))


def uneven_specs(seed: int, n: int = 64, shapes=UNEVEN_SHAPES, coils=(8, 20), accel=(4, 6, 8)):
    """Per-slice (H, W, C, R) of an uneven batch: shape uniform over ``shapes``,
    C ~ U{coils[0]..coils[1]}, R uniform over ``accel``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        H, W = shapes[int(rng.integers(0, len(shapes)))]
        C = int(rng.integers(coils[0], coils[1] + 1))
        R = int(accel[int(rng.integers(0, len(accel)))])
        out.append((H, W, C, R))
    return out


def uneven_inputs(specs, seed0: int, n_center: int = 24, mask_kind: str = "vd", sigma: float = 1e-3):
    """``slice_inputs`` for each (H, W, C, R) of ``specs`` (seed seed0 + i),
    plus the same arrays packed flat in slice order (images, coil data and
    masks concatenated)."""
    sl = [slice_inputs(seed0 + i, H, W, C, R, min(n_center, H // R), mask_kind, sigma)
          for i, (H, W, C, R) in enumerate(specs)]
    packed = {k: np.concatenate([s[k].ravel() for s in sl]) for k in sl[0]}
    return sl, packed
