"""Run the hot kernels alone, for profilers (rocprofv3 --pmc / --kernel-trace).

    python -m paper_2202_14005_amd.profile_kernels [--reps 3] [--what normal,conv,copy]
        [--schedule NAME | --tune]

Workload: the MoDL inference batch (8 slices of 320 x 320, 15 coils, R = 4
variable-density mask with 24 centre lines).  ``normal`` runs one CG solve
of ``reps`` iterations (one CG-fused k_normal launch and one k_cg_update per
iteration, as in the MoDL step; the kernel whose HBM bytes the benchmark's
roofline reports) with the given column schedule, or the autotuner's choice
with --tune, or the default,
``conv`` one 64 -> 64 denoiser layer (k_conv_mid16), ``denoiser`` the
denoiser as MoDL inference runs it (one unroll without CG steps: the fused
first two layers k_conv_first_mid, two k_conv_mid16, k_conv_last), ``backward`` one reverse
pass of the denoiser (input gradient and weight gradients, all five
layers), ``uneven`` ``reps`` CG iterations (one CG-fused normal-operator
launch per matrix size and one CG update each) on the 64-slice uneven batch
({192^2, 256^2, 320^2, 384 x 320}, 8-20 coils, autotuned schedules; its coil
maps exceed the MALL), ``uneven_graph`` ``reps`` replays of the captured
64-slice reconstruction (A^H y, MoDL T = 5, CG-SENSE fallback, judge), for
kernel traces, ``copy`` a device-to-device
copy of 256 MiB (256 MiB read, 256 MiB written) whose counter readings
calibrate FETCH_SIZE and WRITE_SIZE, ``vn`` ``reps`` forward and reverse
passes of the variational network (10 stages, 4 slices of 384 x 320, 15
coils), ``soft`` one soft-SENSE CG solve of ``reps`` iterations (two coil-map
sets, 8 slices of 320 x 320, 15 coils: one search-direction kernel, one
CG-fused k_normal_soft launch with its coil split and one CG update per
iteration).
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2202_14005_amd import ops  # noqa: E402
from synthetic import batch_inputs  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--what", default="normal,conv,copy")
    ap.add_argument("--schedule", default=None)
    ap.add_argument("--tune", action="store_true")
    ap.add_argument("--uneven-schedules", default=None,
                    help="comma-separated column schedules for the uneven batch (one per matrix height), "
                         "instead of the autotuner's choice")
    a = ap.parse_args()
    what = set(a.what.split(","))
    dev = torch.device("cuda", 0)
    B, H, W, C = 8, 320, 320, 15
    d = batch_inputs([2000 + i for i in range(B)], H, W, C, 4, 24, "vd")
    t = lambda x: torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    plan = ops.Plan(H, W, C, B=B, device=dev, network=True)
    x, S, m = t(d["x"]), t(d["S"]), t(d["mask"])
    if a.schedule:
        plan.set_schedule(H, a.schedule)
    elif a.tune:
        plan.autotune(S, m)
    lam = plan.lam(0.05)
    cnn = ops.CNN.init(7, dev)
    a_in = torch.randn(B * H * W * 64, device=dev).to(torch.bfloat16)
    a_out = torch.empty_like(a_in)
    grads = ops.CNNGrads(cnn)
    gz = torch.randn_like(x)
    if "backward" in what:
        plan.cnn_forward(x, cnn)  # activations for the reverse pass
    if "uneven" in what or "uneven_graph" in what:
        from paper_2202_14005_amd.pipeline import Reconstruction
        from synthetic import uneven_inputs, uneven_specs
        specs = uneven_specs(5000)
        _, packed = uneven_inputs(specs, 5000)
        up = ops.Plan([q[0] for q in specs], [q[1] for q in specs], [q[2] for q in specs], device=dev,
                      network=True)
        uS, um = t(packed["S"]), t(packed["mask"])
        uy = up.sense_fwd(t(packed["x"]), uS, um, noise=t(packed["noise"]))
        del packed
        if a.uneven_schedules:
            for name in a.uneven_schedules.split(","):
                up.set_schedule(int(name.split("_")[0][1:]), name)
        else:
            up.autotune(uS, um)
        ua = up.sense_adj(uy, uS, um)
        rec = None
        if "uneven_graph" in what:
            rec = Reconstruction(up, ops.CNN.init(7, dev, last_scale=0.1), uy, uS, um, lam=0.05, T=5, n_cg=10,
                                 ratio=2.0)
            rec.capture()
            rec.replay()
        torch.cuda.synchronize()
        if "uneven" in what:
            up.cg_dc(ua, uS, um, up.lam(0.05), a.reps)
        if rec is not None:
            for _ in range(a.reps):
                rec.replay()
        torch.cuda.synchronize()
        print("uneven schedules:", sorted({up.schedule(b) for b in range(up.B)}), flush=True)
    if "vn" in what:
        # variational network: 10 stages on 4 slices of 384 x 320, 15 coils;
        # forward and reverse pass per rep
        vB, vH, vW = 4, 384, 320
        vd = batch_inputs([7000 + i for i in range(vB)], vH, vW, C, 4, 24, "vd")
        vp = ops.Plan(vH, vW, C, B=vB, device=dev, network=True, vn=True)
        vx, vS, vm = t(vd["x"]), t(vd["S"]), t(vd["mask"])
        vy = vp.sense_fwd(vx, vS, vm, noise=t(vd["noise"]))
        vp.autotune(vS, vm)  # as the benchmark's leg does
        vnet = ops.VarNet.init(vp, seed=1, T=10)
        for _ in range(a.reps):
            vaHy = vp.sense_adj(vy, vS, vm)
            vxT, vst = vnet.forward(vaHy, vS, vm)
            _, vg = vp.mse_grad(vxT, vx)
            vnet.backward(vg, vst, vaHy, vS, vm)
        torch.cuda.synchronize()
        print("vn schedule:", vp.schedule(0), flush=True)
        del vd, vp, vnet, vst
    if "soft" in what:
        from synthetic import soft_batch_inputs
        sd = soft_batch_inputs([2050 + i for i in range(B)], H, W, C, 4, 24, "vd")
        sp = ops.Plan(H, W, C, B=B, device=dev, soft=True)
        sS, sm = t(sd["S"]), t(sd["mask"])
        sy = sp.soft_sense_fwd(t(sd["x"]), sS, sm, noise=t(sd["noise"]))
        saHy = sp.soft_sense_adj(sy, sS, sm)
        del sd
        torch.cuda.synchronize()
        sp.soft_cg_dc(saHy, sS, sm, sp.lam(0.05), a.reps)
        torch.cuda.synchronize()
        print("soft schedule:", sp.schedule(0), flush=True)
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)  # 256 MiB
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    if "normal" in what:
        plan.cg_dc(x, S, m, lam, a.reps)
    for _ in range(a.reps):
        if "conv" in what:
            plan.cnn_layer_forward(2, a_in, cnn, out=a_out)
        if "denoiser" in what:
            # one MoDL unroll with no CG step: the denoiser as inference runs
            # it (fused first two layers, layers 3 and 4, last layer)
            plan.modl_forward(x, S, m, cnn, lam, 1, 0)
        if "backward" in what:
            plan.cnn_backward(x, gz, cnn, grads)
        if "copy" in what:
            dst.copy_(src)
    torch.cuda.synchronize()
    print(f"done: {sorted(what)} x {a.reps}; schedule {plan.schedule(0)}", flush=True)


if __name__ == "__main__":
    main()
