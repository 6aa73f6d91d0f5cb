"""iPALM, the training algorithm the paper names for VarNet (Iterative
Training Algorithms; Variational Network subsection), and the VarNet
parameter constraints, in FP64.  Test infrastructure only: nothing in the
product imports this module.

iPALM (Pock & Sabach's inertial proximal alternating linearized
minimization, cited by the paper) updates blocks theta_j of the weights of a
smooth loss f plus proximal terms g_j.  Step k = 1, 2, ...:

    y_j           = theta_j^k + alpha_k (theta_j^k - theta_j^{k-1})
    theta_j^{k+1} = prox_{tau g_j}( y_j - tau grad_j f(y) )

Readings of what the paper leaves open (it names the algorithm only):

* iPALM's two inertial sequences are taken equal, so the gradient is taken
  at the extrapolated point y, with alpha_k = (k - 1) / (k + 2) (theta^0 =
  theta^1, so the first step is a plain proximal gradient step);
* one fixed step size tau (the learning rate) for all blocks, and all blocks
  updated from one gradient of the mini-batch loss per step;
* the proximal terms are the indicator functions of the original VarNet's
  constraints, so the prox is a projection: each complex filter k_i to zero
  mean and unit Euclidean norm, (v - mean v) / ||v - mean v|| (a filter that
  is zero after removing its mean stays zero); each step size lambda_t to
  lambda_t >= 0; the RBF weights are unconstrained.
"""
from __future__ import annotations

import numpy as np


def alpha(k):
    """Inertia of step k (k >= 1)."""
    return (k - 1.0) / (k + 2.0)


def project_filters(k):
    """Zero mean and unit norm per filter over the last two axes."""
    k = np.asarray(k, dtype=np.complex128)
    v = k - k.mean(axis=(-2, -1), keepdims=True)
    n = np.sqrt(np.sum(np.abs(v) ** 2, axis=(-2, -1), keepdims=True))
    return np.where(n > 0, v / np.where(n > 0, n, 1.0), 0.0)


def project_vn(params):
    """The VarNet constraint projection of a parameter dict {k, w, lam}."""
    return {"k": project_filters(params["k"]),
            "w": np.asarray(params["w"], dtype=np.float64),
            "lam": np.maximum(np.asarray(params["lam"], dtype=np.float64), 0.0)}


def step(theta, theta_prev, k, tau, grad_fn, prox_fn):
    """One iPALM step on a dict of blocks.  grad_fn(y) returns the gradient
    dict at the extrapolated point (complex blocks in the DF^H(1) form, which
    is the real gradient of the real and imaginary parts); prox_fn maps a
    dict to its projection.  Returns (theta^{k+1}, theta^k)."""
    a = alpha(k)
    y = {key: np.asarray(theta[key]) + a * (np.asarray(theta[key]) - np.asarray(theta_prev[key]))
         for key in theta}
    g = grad_fn(y)
    return prox_fn({key: y[key] - tau * np.asarray(g[key]) for key in y}), theta
