"""Build libmrx.so (HIP, gfx950) in-tree.

    python -m paper_2202_14005_amd.build [-j JOBS]

Every source under csrc/ is compiled with hipcc for gfx950 only; the transform
schedule unit (sense_inst.hip) is compiled once per entry of SCHEDULES with
the schedule's parameters as macros, so each length has its kernels
instantiated in a separate object (parallel build, small objects).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmrx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# name, N1, N2, N3, threads per transform T, column tile width, row tile
# height, coil groups per normal-operator workgroup, keep coil values in
# registers (1) or re-read them from L2 (0), and optionally 1 for the
# wave-local normal operator (each wavefront transforms 64 / T columns with
# its own LDS region; G wavefronts per workgroup split the coils), 2 for the
# same with a padded LDS layout; optionally the coil split of CG steps (a
# column tile's coils over that many workgroups, partial outputs added by
# the CG update).
# The first schedule listed for a length is its default; the autotuner
# times all schedules of a length on the normal operator.
SCHEDULES = [
    ("n16_4x4_t4", 4, 4, 1, 4, 16, 16, 1, 1),
    ("n24_4x6_t2", 4, 6, 1, 2, 32, 32, 1, 1),
    ("n32_4x8_t4", 4, 8, 1, 4, 16, 16, 1, 1),
    ("n40_4x10_t2", 4, 10, 1, 2, 32, 32, 1, 1),
    ("n48_4x12_t4", 4, 12, 1, 4, 16, 16, 1, 1),
    ("n64_8x8_t8", 8, 8, 1, 8, 16, 16, 1, 1),
    ("n80_4x4x5_t4", 4, 4, 5, 4, 16, 16, 1, 1),
    ("n96_4x4x6_t8", 4, 4, 6, 8, 16, 16, 1, 1),
    ("n128_4x4x8_t16_w16_g2_rl", 4, 4, 8, 16, 16, 16, 2, 0),
    ("n128_4x4x8_t16_w8_g3_rl", 4, 4, 8, 16, 8, 16, 3, 0),
    ("n128_4x4x8_t16_w16", 4, 4, 8, 16, 16, 16, 1, 1),
    ("n160_4x4x10_t8_w16_g2_rl", 4, 4, 10, 8, 16, 16, 2, 0),
    ("n192_4x4x12_t16_w8_g2_rl", 4, 4, 12, 16, 8, 16, 2, 0),
    ("n192_4x4x12_t16_w16_g2_rl", 4, 4, 12, 16, 16, 16, 2, 0),
    ("n192_4x4x12_t16_w8_g3_rl", 4, 4, 12, 16, 8, 16, 3, 0),
    ("n192_4x4x12_t16_w16", 4, 4, 12, 16, 16, 16, 1, 1),
    ("n256_4x4x16_t16_w8_g2_rl", 4, 4, 16, 16, 8, 16, 2, 0),
    ("n256_4x4x16_t16_w16_g2_rl", 4, 4, 16, 16, 16, 16, 2, 0),
    ("n256_4x4x16_t16_w8_g3_rl", 4, 4, 16, 16, 8, 16, 3, 0),
    ("n256_4x4x16_t16_w16", 4, 4, 16, 16, 16, 16, 1, 1),
    ("n320_4x4x20_t16_w8_g2_rl", 4, 4, 20, 16, 8, 16, 2, 0),
    ("n320_4x4x20_t16_w16_g2_rl", 4, 4, 20, 16, 16, 16, 2, 0),
    ("n320_4x4x20_t16_w16_g3_rl", 4, 4, 20, 16, 16, 16, 3, 0),
    ("n320_4x4x20_t16_w8_g3_rl", 4, 4, 20, 16, 8, 16, 3, 0),
    ("n320_4x4x20_t16_w8_g4_rl", 4, 4, 20, 16, 8, 16, 4, 0),
    ("n320_8x40_t8_w16_g2_rl", 8, 40, 1, 8, 16, 16, 2, 0),
    ("n320_4x4x20_t16_w16", 4, 4, 20, 16, 16, 16, 1, 1),
    ("n384_4x4x24_t16_w8_g2_rl", 4, 4, 24, 16, 8, 16, 2, 0),
    ("n384_4x4x24_t16_w16_g2_rl", 4, 4, 24, 16, 16, 16, 2, 0),
    ("n384_4x4x24_t16_w8_g3_rl", 4, 4, 24, 16, 8, 16, 3, 0),
    ("n384_4x4x24_t16_w16", 4, 4, 24, 16, 16, 16, 1, 1),
    ("n512_4x8x16_t32_w8", 4, 8, 16, 32, 8, 8, 1, 1),
    ("n128_4x4x8_t16_wl_g3", 4, 4, 8, 16, 16, 16, 3, 1, 1),
    ("n128_4x4x8_t16_wl_g4", 4, 4, 8, 16, 16, 16, 4, 1, 1),
    ("n192_4x4x12_t16_wl_g3", 4, 4, 12, 16, 16, 16, 3, 1, 1),
    ("n192_4x4x12_t16_wl_g4", 4, 4, 12, 16, 16, 16, 4, 1, 1),
    ("n256_4x4x16_t16_wl_g3", 4, 4, 16, 16, 16, 16, 3, 1, 1),
    ("n256_4x4x16_t16_wl_g4", 4, 4, 16, 16, 16, 16, 4, 1, 1),
    ("n320_4x4x20_t16_wl_g2", 4, 4, 20, 16, 16, 16, 2, 1, 1),
    ("n320_4x4x20_t16_wl_g3", 4, 4, 20, 16, 16, 16, 3, 1, 1),
    ("n320_4x4x20_t16_wl_g4", 4, 4, 20, 16, 16, 16, 4, 1, 1),
    ("n320_4x4x20_t16_wl_g5", 4, 4, 20, 16, 16, 16, 5, 1, 1),
    ("n384_4x4x24_t16_wl_g3", 4, 4, 24, 16, 16, 16, 3, 1, 1),
    ("n384_4x4x24_t16_wl_g4", 4, 4, 24, 16, 16, 16, 4, 1, 1),
    ("n192_4x4x12_t16_wlp_g4", 4, 4, 12, 16, 16, 16, 4, 1, 2),
    ("n256_4x4x16_t16_wlp_g4", 4, 4, 16, 16, 16, 16, 4, 1, 2),
    ("n320_4x4x20_t16_wlp_g2", 4, 4, 20, 16, 16, 16, 2, 1, 2),
    ("n320_4x4x20_t16_wlp_g4", 4, 4, 20, 16, 16, 16, 4, 1, 2),
    ("n384_4x4x24_t16_wlp_g4", 4, 4, 24, 16, 16, 16, 4, 1, 2),
    ("n192_4x4x12_t16_w16_k3", 4, 4, 12, 16, 16, 16, 1, 1, 0, 3),
    ("n256_4x4x16_t16_w16_k3", 4, 4, 16, 16, 16, 16, 1, 1, 0, 3),
    ("n320_4x4x20_t16_w8_g1_rl", 4, 4, 20, 16, 8, 16, 1, 0),
    ("n320_4x4x20_t16_w16_k2", 4, 4, 20, 16, 16, 16, 1, 1, 0, 2),
    ("n320_4x4x20_t16_w16_k3", 4, 4, 20, 16, 16, 16, 1, 1, 0, 3),
    ("n320_4x4x20_t16_w16_k4", 4, 4, 20, 16, 16, 16, 1, 1, 0, 4),
    ("n320_4x4x20_t16_w16_rl_k3", 4, 4, 20, 16, 16, 16, 1, 0, 0, 3),
    ("n320_4x4x20_t16_w16_g2_rl_k2", 4, 4, 20, 16, 16, 16, 2, 0, 0, 2),
    ("n320_4x4x20_t16_w16_g2_rl_k3", 4, 4, 20, 16, 16, 16, 2, 0, 0, 3),
    ("n320_4x4x20_t16_w8_g2_rl_k2", 4, 4, 20, 16, 8, 16, 2, 0, 0, 2),
    ("n384_4x4x24_t16_w16_k3", 4, 4, 24, 16, 16, 16, 1, 1, 0, 3),
    ("n320_4x4x20_t16_w16_rl_k2", 4, 4, 20, 16, 16, 16, 1, 0, 0, 2),
    ("n320_4x4x20_t16_w16_rl_k4", 4, 4, 20, 16, 16, 16, 1, 0, 0, 4),
    ("n320_4x4x20_t16_w8_rl_k2", 4, 4, 20, 16, 8, 16, 1, 0, 0, 2),
    ("n320_4x4x20_t16_w8_rl_k3", 4, 4, 20, 16, 8, 16, 1, 0, 0, 3),
    ("n320_4x4x20_t16_w8_rl_k4", 4, 4, 20, 16, 8, 16, 1, 0, 0, 4),
    ("n192_4x4x12_t16_w16_rl_k3", 4, 4, 12, 16, 16, 16, 1, 0, 0, 3),
    ("n192_4x4x12_t16_w8_rl_k3", 4, 4, 12, 16, 8, 16, 1, 0, 0, 3),
    ("n256_4x4x16_t16_w16_rl_k3", 4, 4, 16, 16, 16, 16, 1, 0, 0, 3),
    ("n256_4x4x16_t16_w8_rl_k3", 4, 4, 16, 16, 8, 16, 1, 0, 0, 3),
    ("n384_4x4x24_t16_w16_rl_k3", 4, 4, 24, 16, 16, 16, 1, 0, 0, 3),
    ("n384_4x4x24_t16_w8_rl_k3", 4, 4, 24, 16, 8, 16, 1, 0, 0, 3),
]



def _smooth235(n: int) -> bool:
    for f in (2, 3, 5):
        while n % f == 0:
            n //= f
    return n == 1


def generic_schedule(N: int):
    """A default schedule for a length without a tuned one: N = N1 N2 N3
    (each at most 40, composed from the 2/3/4/5 codelets), T threads per
    transform dividing every level's transform count, P = N / T <= 64 points
    per thread, a column tile of WT columns with T WT a whole number of
    wavefronts (the CG dot products reduce over full wavefronts) and at most
    1024 threads, and the normal operator's LDS (N WT complex values plus the
    twiddle and mask tables) within 150 KB.  Preference: fewest points per
    thread (at least 12), power-of-two T, three levels, narrow tiles.
    Coil values are re-read for the conjugate multiply (registers go to the
    points).  None if no decomposition fits."""
    import math
    divs = lambda n: [d for d in range(1, n + 1) if n % d == 0]
    best = None
    for n1 in divs(N):
        for n2 in divs(N // n1):
            n3 = N // n1 // n2
            if n1 < 2 or n2 < 2 or max(n1, n2, n3) > 40:
                continue
            g = math.gcd(math.gcd(N // n1, N // n2), N // n3)
            for t in divs(g):
                P = N // t
                if P > 64 or t > 64:
                    continue
                for wt in (8, 16, 32, 64):
                    if (t * wt) % 64 or t * wt > 1024 or N * wt * 8 + N * 12 > 150 * 1024:
                        continue
                    score = (max(P, 12), 0 if t & (t - 1) == 0 else 1, 0 if n3 > 1 else 1, wt)
                    if best is None or score < best[0]:
                        best = (score, (n1, n2, n3, t, wt))
                    break
    if best is None:
        return None
    n1, n2, n3, t, wt = best[1]
    return (f"n{N}_{n1}x{n2}x{n3}_t{t}_w{wt}_rl_gen", n1, n2, n3, t, wt, wt, 1, 0)


# every even length from 8 to 1024 that factors into 2, 3 and 5 and has no
# tuned schedule above gets a generic one (if a decomposition fits)
_TUNED = {e[1] * e[2] * e[3] for e in SCHEDULES}
GENERIC_SCHEDULES = [g for g in (generic_schedule(n) for n in range(8, 1025, 2)
                                 if _smooth235(n) and n not in _TUNED) if g]
SCHEDULES = SCHEDULES + GENERIC_SCHEDULES


def toep_schedule(L: int):
    """Decomposition of a padded transform length L = 2N for the Toeplitz
    normal operator: L = 2 * N2 * N3 (first radix 2, so that the zero half of
    a padded input is the digit-1 slots), N2, N3 <= 40, T a power of two
    dividing every level's transform count, at most 48 points a thread.
    Preference: fewest points a thread (at least 16), three levels.  Row
    passes use one wavefront a workgroup (64 / T rows), the column pass
    128 / T columns.  None if no decomposition fits."""
    import math
    N = L // 2
    divs = lambda n: [d for d in range(1, n + 1) if n % d == 0]
    best = None
    for n2 in divs(N):
        n3 = N // n2
        if n2 < 2 or n2 > 40 or n3 > 40:
            continue
        g = math.gcd(math.gcd(L // 2, L // n2), L // n3)
        for t in divs(g):
            P = L // t
            if t > 64 or t & (t - 1) or P > 48:
                continue
            score = (max(P, 16), 0 if n3 > 1 else 1, -n3)
            if best is None or score < best[0]:
                best = (score, (n2, n3, t))
    if best is None:
        return None
    n2, n3, t = best[1]
    return (f"t{L}_2x{n2}x{n3}_t{t}", n2, n3, t, max(1, 64 // t), max(1, 128 // t))


# one Toeplitz schedule per padded length 2N of every image length N <= 512
# that has a Cartesian schedule (and a decomposition)
TOEP_SCHEDULES = [g for g in (toep_schedule(2 * n) for n in sorted({e[1] * e[2] * e[3] for e in SCHEDULES})
                              if 2 * n <= 1024) if g]

COMMON_SOURCES = ["api.hip", "ops.hip", "cg_kernels.hip", "autotune.hip", "net.hip", "conv.hip",
                  "conv_wgrad.hip", "vn.hip", "judge.hip"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _extra_sources():
    return [s for s in sorted(os.listdir(CSRC))
            if s.endswith(".hip") and s not in COMMON_SOURCES and s not in ("sense_inst.hip", "toep_inst.hip")]


def _jobs():
    srcs = COMMON_SOURCES + _extra_sources()
    jobs = []
    for s in srcs:
        jobs.append((os.path.join(CSRC, s), os.path.join(BUILD, s.replace(".hip", ".o")), []))
    soft_done = set()
    # the soft normal operator takes 16-column tiles (whole 128-byte rows of
    # the coil maps and images) where the length has a 16-column schedule on
    # the same decomposition; the soft column passes keep the first
    # schedule's tile
    wide = {(e[1], e[2], e[3], e[4]) for e in SCHEDULES
            if e[5] == 16 and not (e[9] if len(e) > 9 else 0)}
    for entry in SCHEDULES:
        name, n1, n2, n3, t, wtc, wtr, g, ks = entry[:9]
        wl = entry[9] if len(entry) > 9 else 0
        kspl = entry[10] if len(entry) > 10 else 1
        # the first column-tiled schedule of each length also carries the
        # length's soft-SENSE kernels
        n = n1 * n2 * n3
        soft = int(not wl and n not in soft_done)
        if soft:
            soft_done.add(n)
        defs = [f"-DMRX_N1={n1}", f"-DMRX_N2={n2}", f"-DMRX_N3={n3}", f"-DMRX_T={t}",
                f"-DMRX_WTC={wtc}", f"-DMRX_WTR={wtr}", f"-DMRX_G={g}", f"-DMRX_KS={ks}",
                f"-DMRX_WL={wl}", f"-DMRX_KSPL={kspl}", f"-DMRX_SOFT={soft}", f'-DMRX_NAME="{name}"']
        if soft and wtc < 16 and (n1, n2, n3, t) in wide:
            defs.append("-DMRX_SOFT_WTN=16")
        jobs.append((os.path.join(CSRC, "sense_inst.hip"), os.path.join(BUILD, f"sched_{name}.o"), defs))
    for name, n2, n3, t, twr, twc in TOEP_SCHEDULES:
        defs = [f"-DMRX_N2={n2}", f"-DMRX_N3={n3}", f"-DMRX_T={t}", f"-DMRX_TWR={twr}", f"-DMRX_TWC={twc}",
                f'-DMRX_NAME="{name}"']
        jobs.append((os.path.join(CSRC, "toep_inst.hip"), os.path.join(BUILD, f"toep_{name}.o"), defs))
    return jobs


def _compile(job):
    src, obj, defs = job
    cmd = [HIPCC, *HIP_FLAGS, *defs, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stderr or "").splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{errs}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Compile every HIP source for gfx950 and link libmrx.so; returns its path."""
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found; set HIPCC")
    os.makedirs(BUILD, exist_ok=True)
    js = _jobs()
    n = jobs or min(16, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=n) as ex:
        objs = list(ex.map(_compile, js))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(objs)} objects", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=None)
    a = ap.parse_args()
    build(a.jobs)
