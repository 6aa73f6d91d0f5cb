"""torch.autograd bindings of the data-consistency layer and of MoDL.

The forward and reverse passes are the library's: ``CGDC.backward`` is the
adjoint CG solve (derivatives of the inversion operator S^{-1}, with S the
self-adjoint A^H A + lambda I, so the reverse pass applies S^{-1} again by the
same CG recipe), and ``MoDLFunction.backward`` walks the unrolls in reverse,
recomputing the denoiser's activations from the stored iterates instead of
keeping them (the paper's checkpointing of derivative data).  torch only
records the tape and holds the tensors.

Complex gradients follow torch's convention for real losses: the gradient of
a complex tensor is dL/dRe + i dL/dIm.
"""
from __future__ import annotations

import torch

from .ops import CNN, CNNGrads, Plan


def _lam_grad(lam, g):
    """Reduce the per-slice gradient g [B] to the shape of ``lam``."""
    if not isinstance(lam, torch.Tensor):
        return None
    if lam.numel() == 1:
        return g.sum().reshape(lam.shape).to(lam.dtype)
    return g.reshape(lam.shape).to(lam.dtype)


class CGDC(torch.autograd.Function):
    """x = (A^H A + lambda I)^{-1} (aHy + lambda z) by n_iter CG steps from 0."""

    @staticmethod
    def forward(ctx, aHy, z, lam, plan: Plan, S, mask, n_iter: int):
        lt = plan.lam(lam.detach() if isinstance(lam, torch.Tensor) else lam)
        zc = z.detach().contiguous() if z is not None else None
        x = plan.cg_dc(aHy.detach().contiguous(), S, mask, lt, n_iter, z=zc)
        ctx.plan, ctx.S, ctx.mask, ctx.n_iter, ctx.lam = plan, S, mask, n_iter, lam
        ctx.save_for_backward(x, zc, lt)
        return x

    @staticmethod
    def backward(ctx, gx):
        x, z, lt = ctx.saved_tensors
        need_a, need_z, need_l = ctx.needs_input_grad[:3]
        if not (need_a or need_z or need_l):
            return (None,) * 7
        ga, gz, gl = ctx.plan.cg_dc_backward(gx.contiguous(), x, ctx.S, ctx.mask, lt, ctx.n_iter, z=z,
                                             need_z=need_z and z is not None, need_lam=need_l)
        glam = _lam_grad(ctx.lam, gl) if need_l else None
        return (ga if need_a else None), (gz if need_z else None), glam, None, None, None, None


def cg_dc(plan: Plan, aHy, S, mask, lam, n_iter: int, z=None):
    """Differentiable data-consistency solve (w.r.t. aHy, z and lam)."""
    return CGDC.apply(aHy, z, lam, plan, S, mask, n_iter)


class MoDLFunction(torch.autograd.Function):
    """x^T of eq. update_modl from x^0 = aHy, differentiable w.r.t. aHy,
    lambda and the ten denoiser parameters (weights and biases, layer order)."""

    @staticmethod
    def forward(ctx, aHy, lam, plan: Plan, cnn: CNN, S, mask, T: int, n_cg: int, *params):
        lt = plan.lam(lam.detach() if isinstance(lam, torch.Tensor) else lam)
        a = aHy.detach().contiguous()
        x, states = plan.modl_forward(a, S, mask, cnn, lt, T, n_cg, states=True)
        ctx.plan, ctx.cnn, ctx.S, ctx.mask, ctx.T, ctx.n_cg, ctx.lam = plan, cnn, S, mask, T, n_cg, lam
        ctx.save_for_backward(a, states, lt)
        return x

    @staticmethod
    def backward(ctx, gx):
        a, states, lt = ctx.saved_tensors
        grads = CNNGrads(ctx.cnn)
        gl, ga = ctx.plan.modl_backward(gx.contiguous(), states, a, ctx.S, ctx.mask, ctx.cnn, lt, ctx.T,
                                        ctx.n_cg, grads, need_aHy=ctx.needs_input_grad[0])
        glam = _lam_grad(ctx.lam, gl) if ctx.needs_input_grad[1] else None
        return (ga, glam, None, None, None, None, None, None) + tuple(grads.params())


class MoDLNet(torch.nn.Module):
    """MoDL as a torch module: fp32 master weights are ``nn.Parameter``s
    (channels 2-64-64-64-64-2), lambda is a fixed float or, with
    ``learn_lam=True``, a learnable scalar parameter."""

    def __init__(self, plan: Plan, T=5, n_cg=10, lam=0.05, learn_lam=False, seed=7):
        super().__init__()
        if not plan.network:
            raise ValueError("MoDLNet needs a plan created with network=True")
        init = CNN.init(seed=seed, device=plan.device)
        self.weights = torch.nn.ParameterList([torch.nn.Parameter(w.clone()) for w in init.w])
        self.biases = torch.nn.ParameterList([torch.nn.Parameter(b.clone()) for b in init.b])
        self.lam = (torch.nn.Parameter(torch.tensor([float(lam)], device=plan.device)) if learn_lam
                    else float(lam))
        self.plan, self.T, self.n_cg = plan, int(T), int(n_cg)
        self.cnn = CNN(list(self.weights), list(self.biases))

    def forward(self, y, S, mask):
        """Reconstruct from k-space y (x^0 = A^H y computed here)."""
        return self.forward_from_adjoint(self.plan.sense_adj(y, S, mask), S, mask)

    def forward_from_adjoint(self, aHy, S, mask):
        """Reconstruct from a precomputed A^H y (differentiable w.r.t. it)."""
        params = []
        for w, b in zip(self.weights, self.biases):
            params += [w, b]
        return MoDLFunction.apply(aHy, self.lam, self.plan, self.cnn, S, mask, self.T, self.n_cg, *params)
