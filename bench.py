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

DESCRIPTIONS = {
    "channel2d": "channel2d: layered two-phase Poiseuille channel, 1024x256 jittered P1 mesh, D2Q9, "
                 "density ratio 1000, viscosity ratio 50",
    "droplet2d": "droplet2d: static drop, 64x64 periodic jittered P1 mesh, D2Q9, density ratio 10",
    "rt2d": "rt2d: Rayleigh-Taylor, 1024x4096 jittered P1 mesh between walls, D2Q9, Atwood 0.5",
    "droplet3d": "droplet3d: static drop, 128^3 periodic jittered Kuhn-tet mesh, D3Q19, density ratio 100",
    "ensemble2d": "ensemble2d: 64 independent periodic drops, sides 32..512, density ratios 1..1000, D2Q9",
    "translate2d": "translate2d: drop carried by u0 = 0.02 through a 128x128 periodic jittered P1 mesh, D2Q9, "
                   "density ratio 100",
}


def kernel_bytes(cls: str, *, Q: int, D: int, W: int, NB: int, s: int, sp: int, dev: bool,
                 first_frac: float = 0.0, K: int = 0) -> float:
    """Algorithmic HBM bytes per node row of one launch of a kernel class:
    every operand read or written once (gathers of neighbour values served
    by cache), pattern = 4-byte column index per off-diagonal slot (slot 0
    is the row itself).  s = operator/vector value size, sp = stored
    population size, dev = deviation storage with two 4-byte node
    references, where streaming works on differences to the row's own value
    and needs no diagonal coefficients.  K = CG iterations (every
    iteration's direction is stored and x formed once, by cg_x)."""
    NP = 2 * (Q - 1)
    P = 2 * Q
    pat = (W - 1) * 4
    ref = 8 if dev else 0
    if cls == "stream":
        return NP * sp + ref + pat + NB * (W - 1 if dev else W) * s + NP * s
    if cls == "cg_init":  # read rhs, write r (x_0 = rhs / m is formed again by cg_x)
        return 2 * NP * s + pat + W * s + s
    qrec = W >= 15  # the CG carries q = M p by its own recurrence on the 3-D widths
    if cls == "cg_a":
        if qrec:  # read r, p, q; write p, q (the first iteration reads r only)
            return (5 - 2 * first_frac) * NP * s + pat + W * s + s
        # read r, p_old; write p_new (p_old unread on the first iteration)
        return (3 - first_frac) * NP * s + pat + W * s + s
    if cls == "cg_b":
        if qrec:  # read q, r; write r (own rows only)
            return 3 * NP * s + s
        # read p, r; write r (M p formed again from neighbour values of p)
        return 3 * NP * s + pat + W * s + s
    if cls == "cg_x":
        # x = rhs / m + sum_k alpha_k p_k: read rhs, 1/m and the K directions, write x
        return (2 + K) * NP * s + s
    if cls == "cheb_first":
        return 3 * NP * s + pat + W * s + s
    if cls == "cheb":
        return 4 * NP * s + pat + W * s + s
    if cls == "lumped":
        return 2 * NP * s + s
    if cls == "moments":
        return Q * sp + (Q - 1) * s + 4 + s + ref // 2
    if cls == "grad":
        return s + pat + D * W * s + D * s
    if cls == "div":
        return D * s + s + pat + D * W * s + (1 + D) * s
    if cls == "collide":
        return 2 * P * sp + NP * s + (2 + 2 * D) * s + pat + D * W * s + s + 4 + (D + 1) * s + 2 * ref
    return 0.0


def cpu_baseline(workload, target_s: float = 15.0, mass_mode: int = 0):
    """The FP64 oracle, as it stands, on the same workload for ~target_s of
    CPU time (lumped mass when the device runs lumped, else its exact
    consistent-mass solve)."""
    from oracle import oracle as O
    inst = workload.instances[0]
    o = O.Oracle(inst.mesh, workload.lattice, inst.phys, mass_mode=1 if mass_mode == 1 else 0)
    o.init(inst.rho0, inst.u0, inst.p0)
    t0 = time.perf_counter()
    o.step(1)
    per = time.perf_counter() - t0
    more = max(1, int(target_s / max(per, 1e-3)) - 1)
    o.step(more)
    secs = time.perf_counter() - t0
    steps = 1 + more
    N = inst.mesh["xyz"].shape[0]
    out = dict(value=N * 2 * workload.lattice * steps / secs, unit="NPU/s", cores=1, kind="oracle",
               sample=f"first {steps} steps of the same {N}-node workload (plain FP64 C oracle, 1 thread, "
                      f"{secs:.1f} s)")
    return out, o, steps


def measured_traffic(workload: str, precision: str, mass_mode: int, kernel: str, name: str | None):
    """HBM bytes per launch of kernel `name` (class `kernel`) from the
    committed rocprofv3 counter summary (FETCH_SIZE and WRITE_SIZE scaled by
    their copy-kernel calibration), or None when no summary covers this
    configuration and kernel or the device sources changed since the
    counters were taken."""
    from paper_1608_01906_amd.profiling import device_source_hash, lookup_traffic
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic_{precision}_mass{mass_mode}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if device_source_hash() != rec["kernel_source_sha256_16"]:
        return None
    return lookup_traffic(rec, kernel, name)


def run_gpu(w, precision, steps, warmup, prof_steps, mass_mode=0, workload="channel2d", node_order=0):
    import torch
    from paper_1608_01906_amd import felbm
    N = w.n_nodes
    P = 2 * w.lattice
    ctx = felbm.from_workload(w, precision=precision, device="cuda:0", mass_mode=mass_mode, node_order=node_order)
    info = ctx.layout_info()
    ctx.step(warmup)
    ctx.sync(allow_notconv=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    status = "ok"
    try:
        ctx.sync(allow_notconv=True)
    except felbm.FelError as e:  # the state went non-finite; the timing still stands
        status = str(e)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    # event-timed pass: the same step graph with an event pair around every kernel
    ctx.profile(True)
    ctx.step(prof_steps)
    try:
        prof = ctx.profile_read()
    except felbm.FelError:
        prof = ctx.profile_read()
    ctx.profile(False)
    s = 8 if precision == "fp64" else 4
    sp = {"fp64": 8, "fp32": 4, "fp32_fp16": 2}[precision]
    D = 2 if w.lattice == 9 else 3
    NB = 5 if D == 2 else 9
    kern = {}
    for name, (cnt, ms) in prof.items():
        if cnt == 0:
            continue
        first = (1.0 / info["cg_iters"]) if name == "cg_a" and info["cg_iters"] else 0.0
        b = kernel_bytes(name, Q=w.lattice, D=D, W=info["ell_width"], NB=NB, s=s, sp=sp,
                         dev=precision != "fp64", first_frac=first, K=info["cg_iters"]) * N
        if name == "cheb":
            # one first launch (gathers rhs, writes x0 and x1) per K launches
            K = info["cg_iters"]
            kw = dict(Q=w.lattice, D=D, W=info["ell_width"], NB=NB, s=s, sp=sp, dev=precision != "fp64")
            b = (kernel_bytes("cheb_first", **kw) + (K - 1) * kernel_bytes("cheb", **kw)) / K * N
        avg_ms = ms / cnt
        kern[name] = dict(launches=cnt, avg_us=round(avg_ms * 1e3, 3), total_ms=round(ms, 3),
                          bytes_per_launch=int(b), gbs=round(b / (avg_ms * 1e-3) / 1e9, 1))
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    dk = kern[dom]
    sched = ctx.tuning()
    dom_name = None
    if dom in ("cg_init", "cg_a", "cg_b", "cheb"):
        from paper_1608_01906_amd.profiling import solver_kernel_name
        b, sg = sched[dom]
        dom_name = solver_kernel_name(dom, precision, info["ell_width"], 2 * (w.lattice - 1), b, sg == 2,
                                      sched.get("fused") == 2)
    step_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in kern.values()) / prof_steps
    res = dict(value=N * P * steps / secs, ms_per_step=secs / steps * 1e3, cg_iters=info["cg_iters"],
               status=status,
               roofline=dict(bound="hbm", kernel=dom, achieved=dk["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=round(dk["gbs"] / HBM_PEAK_GBS, 4),
                             traffic=measured_traffic(workload, precision, mass_mode, dom, dom_name),
                             bytes_per_launch=dk["bytes_per_launch"], avg_launch_us=dk["avg_us"],
                             kernel_instance=dom_name),
               step_algorithmic_gbs=round(step_bytes / (secs / steps) / 1e9, 1),
               step_frac=round(step_bytes / (secs / steps) / 1e9 / HBM_PEAK_GBS, 4),
               kernels=kern,
               schedule=dict({k: dict(batch=v[0], staging=("direct", "lds")[v[1] - 1])
                              for k, v in sched.items() if k in ("cg_init", "cg_a", "cg_b", "cheb") and k in kern},
                             reductions="fused" if sched.get("fused") == 2 else "finalize launches"),
               halo=dict(max=info["halo_max"], mean=round(info["halo_mean"], 1)),
               event_ms_per_step=round(sum(v["total_ms"] for v in kern.values()) / prof_steps, 4))
    return res, ctx


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000, help="timed steps (the workload's full length)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp32_fp16"],
                    help="precision of the headline value (the FP64 plain path is measured beside it)")
    ap.add_argument("--profile-steps", type=int, default=100, help="steps of the event-timed pass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison run")
    ap.add_argument("--workload", default="channel2d", choices=sorted(DESCRIPTIONS),
                    help="workload (default: the 1024 x 256 layered channel)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="first copy this many MiB device-to-device (HBM counter calibration)")
    ap.add_argument("--no-chebyshev", action="store_true",
                    help="skip the run with the mass matrix solved by Chebyshev iteration")
    ap.add_argument("--no-lumped", action="store_true",
                    help="skip the run with the lumped mass matrix (the paper's own approximation)")
    ap.add_argument("--mass-mode", type=int, default=0, choices=[0, 1, 2],
                    help="mass solve of the headline run: 0 consistent (CG), 1 lumped, 2 consistent (Chebyshev)")
    ap.add_argument("--node-order", type=int, default=0, choices=[0, 1],
                    help="device row order: 0 the workload's node order, 1 Z-order curve")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the channel would shard as slabs along x with one-layer halos; see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    from paper_1608_01906_amd.inputs import WORKLOADS
    from tests._parity import compare_fields

    if args.copy_probe:
        # a plain device copy of known size, for calibrating the HBM counters
        import torch
        nb = int(args.copy_probe * 2 ** 20)
        a = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
    w = WORKLOADS[args.workload]()
    inst = w.instances[0]
    N = w.n_nodes
    P = 2 * w.lattice
    head, ctx_head = run_gpu(w, args.precision, args.steps, args.warmup, args.profile_steps,
                             mass_mode=args.mass_mode, workload=args.workload, node_order=args.node_order)
    mass = {0: f"consistent, CG x{head['cg_iters']}", 1: "lumped",
            2: f"consistent, Chebyshev x{head['cg_iters']}"}[args.mass_mode]
    out = {
        "metric": "node-population updates/s (NPU/s)",
        "value": head["value"],
        "unit": "NPU/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_fp16": "f32 (f16 storage)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS.get(args.workload, w.name), "instances": len(w.instances),
                   "nodes": N, "populations": P, "precision": args.precision,
                   "mass": mass, "dt": inst.phys.dt,
                   "node_order": ("workload", "z-curve")[args.node_order]},
        "roofline": head["roofline"],
        "step_algorithmic_gbs": head["step_algorithmic_gbs"],
        "step_frac": head["step_frac"],
        "kernels": head["kernels"],
        "schedule": head["schedule"],
        "halo": head["halo"],
        "event_ms_per_step": head["event_ms_per_step"],
        "status": head["status"],
    }
    ctx64 = None
    if not args.no_fp64 and args.precision != "fp64":
        r64, ctx64 = run_gpu(w, "fp64", args.steps, args.warmup, args.profile_steps, mass_mode=args.mass_mode,
                             workload=args.workload, node_order=args.node_order)
        out["fp64_plain"] = {k: r64[k] for k in ("value", "ms_per_step", "roofline", "step_algorithmic_gbs",
                                                 "step_frac", "event_ms_per_step")}
        out["speedup_vs_fp64_plain"] = head["value"] / r64["value"]
    if not args.no_chebyshev and args.mass_mode != 2:
        rch, _ = run_gpu(w, args.precision, args.steps, args.warmup, args.profile_steps, mass_mode=2,
                         workload=args.workload, node_order=args.node_order)
        out["chebyshev_solve"] = {k: rch[k] for k in ("value", "ms_per_step", "roofline", "step_algorithmic_gbs",
                                                      "step_frac", "event_ms_per_step", "schedule")}
    if not args.no_lumped and args.mass_mode != 1:
        rlu, _ = run_gpu(w, args.precision, args.steps, args.warmup, args.profile_steps, mass_mode=1,
                         workload=args.workload, node_order=args.node_order)
        out["lumped_mass"] = {k: rlu[k] for k in ("value", "ms_per_step", "roofline", "step_algorithmic_gbs",
                                                  "step_frac", "event_ms_per_step")}
    if not args.no_cpu_baseline:
        from paper_1608_01906_amd import felbm
        cb, orc, s_steps = cpu_baseline(w, mass_mode=args.mass_mode)
        out["cpu_baseline"] = cb
        ref = orc.fields()
        errs = {}
        for prec in [args.precision] + ([] if args.no_fp64 or args.precision == "fp64" else ["fp64"]):
            c = felbm.from_workload(w, precision=prec, device="cuda:0", mass_mode=args.mass_mode,
                                    node_order=args.node_order)
            c.step(s_steps)
            c.sync(allow_notconv=True)
            errs[prec] = {k: float(f"{v:.3e}") for k, v in compare_fields(c.read_fields(0), ref, inst).items()}
        out["error_vs_oracle"] = dict(steps=s_steps, norm="max |dev - oracle| / max(|oracle|, floor)", **errs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
