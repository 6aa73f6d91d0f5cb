"""Conjugate gradients and the inversion operator S^{-1} (MoDL subsection:
the generic inversion of a parametrised self-adjoint positive-definite
S_lambda, its derivatives D_y S^{-1} = S^{-1} and
D_lambda S^{-1} = -S^{-1} o D_lambda S, applied by CG as proposed for MoDL).

Readings of points the paper leaves open:

* Textbook Hestenes-Stiefel CG with x0 = 0 and a fixed iteration count n; no
  tolerance stop.  Only exact breakdown is guarded: when rho = 0 or
  Re<p, S p> <= 0 the iteration stops and keeps the current x.
* Inner product <u, v> = sum conj(u) v over one slice; each slice of a batch
  has its own scalars.
* The backward pass of the truncated forward solve is defined as S^{-1}
  applied by the same CG recipe (same n, x0 = 0) to the incoming gradient.
"""
from __future__ import annotations

import numpy as np

from . import sense


def _dot(u, v):
    return np.sum(np.conj(u) * v, axis=(-2, -1))  # per slice


def cg(apply_S, b, n_iter):
    """Solve S x = b slice by slice with n_iter CG steps, x0 = 0.

    Returns (x, rho_hist) where rho_hist[b, k] = ||r_k||^2 for k = 0..n_iter.
    """
    b = np.asarray(b, dtype=np.complex128)
    B = b.shape[0]
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = _dot(r, r).real
    hist = np.zeros((B, n_iter + 1))
    hist[:, 0] = rho
    active = rho > 0
    for k in range(n_iter):
        q = apply_S(p)
        pq = _dot(p, q).real
        active = active & (pq > 0)
        alpha = np.where(active, rho / np.where(active, pq, 1.0), 0.0)
        x = x + alpha[:, None, None] * p
        r = r - alpha[:, None, None] * q
        rho_new = _dot(r, r).real
        beta = np.where(active & (rho > 0), rho_new / np.where(rho > 0, rho, 1.0), 0.0)
        p = np.where(active[:, None, None], r + beta[:, None, None] * p, p)
        rho = np.where(active, rho_new, rho)
        active = active & (rho > 0)
        hist[:, k + 1] = rho
    return x, hist


def normal_op(S, m, lam):
    return lambda v: sense.sense_normal(v, S, m, lam)


def cg_dc(aHy, z, S, m, lam, n_iter):
    """Data-consistency block of eq. update_modl:
    x = (A^H A + lambda I)^{-1} (A^H y + lambda z), computed by n_iter CG steps.
    z = None means z = 0 (plain Tikhonov CG-SENSE)."""
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    b = np.asarray(aHy, dtype=np.complex128)
    if z is not None:
        b = b + lam[:, None, None] * np.asarray(z, dtype=np.complex128)
    return cg(normal_op(S, m, lam), b, n_iter)


def cg_sense(y, S, m, lam, n_iter):
    """Plain CG-SENSE: x = (A^H A + lambda I)^{-1} A^H y."""
    return cg_dc(sense.sense_adj(y, S, m), None, S, m, lam, n_iter)


def cg_dc_backward(gx, x, z, S, m, lam, n_iter):
    """Reverse-mode pass of ``cg_dc``.

    With b = a + lambda z, S = A^H A + lambda I, x = S^{-1} b and upstream
    gradient g (in the DF^H(1) form: real part = d/dRe, imaginary = d/dIm):
      v = S^{-1} g  (S is self-adjoint),
      dL/da = v,  dL/dz = lambda v,  dL/dlambda = Re<v, z - x>.
    The last follows from differentiating (A^H A + lambda I) x = a + lambda z
    in lambda: dx = S^{-1}(z - x) dlambda.
    Returns (g_a, g_z, g_lambda[B]).
    """
    lam = np.asarray(lam, dtype=np.float64).reshape(-1)
    v, _ = cg(normal_op(S, m, lam), gx, n_iter)
    zz = 0.0 if z is None else np.asarray(z, dtype=np.complex128)
    g_lam = _dot(v, zz - np.asarray(x, dtype=np.complex128)).real
    return v, lam[:, None, None] * v, g_lam
