"""Batched reconstruction with fallback: k-space to image for one (possibly
uneven) batch of slices, run eagerly or replayed from one captured HIP graph.

Steps, all in the library's kernels on one stream:

1. x0 = A^H y (SENSE adjoint);
2. MoDL: T unrolls of [denoiser, CG data consistency] (eq. update_modl);
3. plain Tikhonov CG-SENSE, x_cg = (A^H A + lambda_cg I)^{-1} A^H y, the
   reconstruction the method reduces to without its learned prior;
4. the judge: per slice keep the MoDL image unless it is non-finite, flagged,
   or its data-consistency residual ||A^H A x - A^H y|| exceeds ``ratio``
   times that of x_cg; otherwise return x_cg;
5. the per-slice status words of this run (cleared at its start) are copied
   out.

Slices of different (H, W, C) are grouped by matrix size inside the plan; each
operator launches one kernel per group and one element-wise kernel over the
whole batch, so a whole reconstruction is a fixed sequence of launches that a
graph replays with no host work.  Column-transform schedules come from the
plan (its autotuner, or a saved tuning cache loaded before the plan was made).
"""
from __future__ import annotations

import torch

from .ops import CNN, Plan


class Reconstruction:
    """MoDL + CG-SENSE fallback over the static input tensors ``y``, ``S``,
    ``mask`` (packed or batched as for ``Plan``).  Results are written into
    ``self.out`` (image), ``self.choice`` (int32 [B], 1 = fallback taken) and
    ``self.flags`` (int32 [B], status bits of this run); ``self.x_net`` and
    ``self.x_cg`` hold the two candidates.

    The tensors' addresses are baked into the captured graph: refill them in
    place between replays.  Updated denoiser weights are repacked before the
    next replay (the packed copy lives at a fixed place in the workspace)."""

    def __init__(self, plan: Plan, cnn: CNN, y, S, mask, lam=0.05, T=5, n_cg=10, lam_cg=None,
                 n_cg_fallback=None, ratio=2.0):
        if not plan.network:
            raise ValueError("Reconstruction needs a plan created with network=True")
        if not ratio > 0:
            raise ValueError("ratio must be positive")
        plan._coil(y, "y"); plan._coil(S, "S"); plan._mask(mask, "mask")
        self.plan, self.cnn = plan, cnn
        self.y, self.S, self.mask = y, S, mask
        self.T, self.n_cg = int(T), int(n_cg)
        self.n_fb = int(n_cg_fallback if n_cg_fallback is not None else n_cg)
        self.ratio = float(ratio)
        self.lam = plan.lam(lam)
        self.lam_cg = plan.lam(lam_cg if lam_cg is not None else lam)
        self.aHy = plan._empty_img()
        self.x_net = plan._empty_img()
        self.x_cg = plan._empty_img()
        self.out = plan._empty_img()
        self.choice = torch.zeros(plan.B, dtype=torch.int32, device=plan.device)
        self.flags = torch.zeros(plan.B, dtype=torch.int32, device=plan.device)
        self.graph = None

    def _enqueue(self):
        p = self.plan
        p.clear_status()
        p.sense_adj(self.y, self.S, self.mask, out=self.aHy)
        p.modl_forward(self.aHy, self.S, self.mask, self.cnn, self.lam, self.T, self.n_cg, out=self.x_net)
        p.cg_dc(self.aHy, self.S, self.mask, self.lam_cg, self.n_fb, out=self.x_cg)
        p.dc_judge(self.x_net, self.x_cg, self.aHy, self.S, self.mask, self.ratio, out=self.out,
                   choice=self.choice)
        p.status(out=self.flags)

    def run(self):
        """Eager run on the current stream; returns ``self.out``."""
        self.plan.set_weights(self.cnn)
        self._enqueue()
        return self.out

    def capture(self):
        """Record one reconstruction into a graph (after a warm-up run on a
        side stream, as graph capture requires)."""
        dev = self.plan.device
        self.plan.set_weights(self.cnn)  # packing stays outside the graph
        cur = torch.cuda.current_stream(dev)
        side = torch.cuda.Stream(dev)
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            self._enqueue()
        cur.wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._enqueue()
        self.graph = g
        return g

    def replay(self):
        """Replay the captured reconstruction; returns ``self.out``."""
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.plan.set_weights(self.cnn)  # no-op unless the weights changed
        self.graph.replay()
        return self.out
