#!/usr/bin/env python
"""Throughput of the FE lattice Boltzmann step on one MI355X.

Workload: the layered two-phase Poiseuille channel, 1024 x 256 jittered P1
mesh (262,144 nodes, D2Q9, density ratio 1000, viscosity ratio 50), seeded
synthetic inputs resident in HBM before timing.  A step is one full time
step: streaming right-hand side, CG solve on the mass matrix, walls and
moments, recovery of the derivatives, fused collision.

Metric: node-population updates per second, NPU/s = nodes * 2Q * steps / s.
Prints one JSON line with the roofline of the dominant kernel (HIP events
on the library's stream, algorithmic bytes per launch) and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def kernel_bytes(cls: str, *, Q: int, D: int, W: int, NB: int, s: int, sp: int, first_frac: float = 0.0) -> float:
    """Algorithmic HBM bytes per node row of one launch of a kernel class:
    every operand read or written once (gathers of neighbour values served
    by cache), pattern = 4-byte column index per slot."""
    NP = 2 * (Q - 1)
    P = 2 * Q
    pat = W * 4
    if cls == "stream":
        return NP * sp + (2 * sp if sp != 8 and sp != 4 else 0) + pat + NB * W * s + NP * s
    if cls == "cg_init":
        return 3 * NP * s + pat + W * s + s
    if cls == "cg_a":
        return (3 - first_frac) * NP * s + pat + W * s + s
    if cls == "cg_b":
        return 5 * NP * s + pat + W * s + s
    if cls == "lumped":
        return 2 * NP * s + s
    if cls == "moments":
        return Q * sp + (Q - 1) * s + 4 + s
    if cls == "grad":
        return s + pat + D * W * s + D * s
    if cls == "div":
        return D * s + s + pat + D * W * s + (1 + D) * s
    if cls == "collide":
        return 2 * P * sp + NP * s + (2 + 2 * D) * s + pat + D * W * s + s + 4 + (D + 1) * s
    return 0.0


def cpu_baseline(workload, target_s: float = 15.0):
    from oracle import oracle as O
    inst = workload.instances[0]
    o = O.Oracle(inst.mesh, workload.lattice, inst.phys)
    o.init(inst.rho0, inst.u0, inst.p0)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter()
    per = t1 - t0
    more = max(1, int(target_s / max(per, 1e-3)) - 1)
    o.step(more)
    t2 = time.perf_counter()
    steps = 1 + more
    secs = t2 - t0
    N = inst.mesh["xyz"].shape[0]
    return dict(value=N * 2 * workload.lattice * steps / secs, unit="NPU/s", cores=1, kind="oracle",
                sample=f"{steps} steps of the same {N}-node workload, plain FP64 C oracle, 1 thread, "
                       f"{secs:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "fp32_fp16"])
    ap.add_argument("--profile-steps", type=int, default=0, help="steps of the event-timed pass (default: --steps)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the channel would shard as slabs along x with one-layer halos; see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1608_01906_amd import felbm
    from paper_1608_01906_amd.inputs import channel2d

    w = channel2d()
    inst = w.instances[0]
    N = inst.mesh["xyz"].shape[0]
    Q = w.lattice
    P = 2 * Q
    ctx = felbm.from_workload(w, precision=args.precision, device="cuda:0")
    info = ctx.layout_info()
    ctx.step(args.warmup)
    ctx.sync(allow_notconv=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps)
    ctx.sync(allow_notconv=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    secs = t1 - t0
    value = N * P * args.steps / secs

    # event-timed pass (same kernels, one launch at a time) for the roofline
    psteps = args.profile_steps or args.steps
    ctx.profile(True)
    ctx.step(psteps)
    prof = ctx.profile_read()
    ctx.profile(False)
    s = 8 if args.precision == "fp64" else 4
    sp = {"fp64": 8, "fp32": 4, "fp32_fp16": 2}[args.precision]
    D = 2
    W = info["ell_width"]
    NB = 5
    kern = {}
    for name, (cnt, ms) in prof.items():
        if cnt == 0:
            continue
        frac_first = (1.0 / info["cg_iters"]) if name == "cg_a" and info["cg_iters"] else 0.0
        b = kernel_bytes(name, Q=Q, D=D, W=W, NB=NB, s=s, sp=sp, first_frac=frac_first) * N
        avg_ms = ms / cnt
        kern[name] = dict(launches=cnt, avg_us=avg_ms * 1e3, total_ms=ms, bytes_per_launch=b,
                          gbs=b / (avg_ms * 1e-3) / 1e9)
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    dk = kern[dom]
    step_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in kern.values()) / psteps
    roofline = dict(bound="hbm", kernel=dom, achieved=round(dk["gbs"], 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(dk["gbs"] / HBM_PEAK_GBS, 4), traffic=None,
                    bytes_per_launch=int(dk["bytes_per_launch"]), avg_launch_us=round(dk["avg_us"], 2))
    prof_step_ms = sum(v["total_ms"] for v in kern.values()) / psteps

    out = {
        "metric": "node-population updates/s (NPU/s)",
        "value": value,
        "unit": "NPU/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_fp16": "f32 (f16 storage)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "channel2d 1024x256 jittered P1, D2Q9, density ratio 1000, viscosity ratio 50",
                   "nodes": N, "populations": P, "precision": args.precision,
                   "mass": "consistent, CG x%d" % info["cg_iters"], "dt": inst.phys.dt},
        "roofline": roofline,
        "step_hbm_gbs": round(step_bytes / (secs / args.steps) / 1e9, 1),
        "kernels": {k: {kk: round(vv, 3) if isinstance(vv, float) else vv for kk, vv in v.items()}
                    for k, v in kern.items()},
        "profiled_ms_per_step": prof_step_ms,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
