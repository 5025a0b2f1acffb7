#!/usr/bin/env python
"""Throughput of the FE lattice Boltzmann step on one MI355X.

Workload (default): the batched ensemble, 64 independent periodic D2Q9
droplets on jittered P1 meshes with sides drawn in 32..512 (seeded, 6.58 M
nodes in all) and density ratios log-uniform in 1..1000, advanced together:
every launch covers all instances and each step is one replay of a captured
graph.  Seeded synthetic inputs are resident in HBM before timing.  A step
is one full time step: streaming right-hand side, CG solve on the mass
matrix, moments, recovery of the derivatives, fused collision.

Metric: node-population updates per second, NPU/s = nodes * 2Q * steps / s,
for the FP32 path (scaled-deviation storage, FP64 CG dots and sums) with the
FP64 plain path on the same meshes beside it.  Prints one JSON line with
the roofline of the dominant kernel (HIP events on the library's stream,
algorithmic bytes per launch), the whole step's fraction of the HBM
roofline, the CPU oracle timed on the first steps of the same workload, and
every instance's error against the oracle after those steps.
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

# Device row order of the headline by workload: the Z-order curve (tiles of
# 16 x 16 lattice nodes, halos of ~70 rows instead of two grid rows) where
# the LDS-staged kernels then beat direct gathers: the batched drops and the
# 4.2 M-node Rayleigh-Taylor mesh.  The channel's fused kernels gather
# directly and the 3-D streaming kernel has no staged form, so those keep
# the workload's order.
ZORDER_DEFAULT = {"ensemble2d": 1, "rt2d": 1}

DESCRIPTIONS = {
    "channel2d": "channel2d: layered two-phase Poiseuille channel, 1024x256 jittered P1 mesh, D2Q9, "
                 "density ratio 1000, viscosity ratio 50",
    "droplet2d": "droplet2d: static drop, 64x64 periodic jittered P1 mesh, D2Q9, density ratio 10",
    "rt2d": "rt2d: Rayleigh-Taylor, 1024x4096 jittered P1 mesh between walls, D2Q9, Atwood 0.5",
    "droplet3d": "droplet3d: static drop, 128^3 periodic jittered Kuhn-tet mesh, D3Q19, density ratio 100",
    "ensemble2d": "ensemble2d: 64 independent periodic drops, sides 32..512, density ratios 1..1000, D2Q9",
    "translate2d": "translate2d: drop carried by u0 = 0.02 through a 128x128 periodic jittered P1 mesh, D2Q9, "
                   "density ratio 100",
    "pipe3d": "pipe3d: concurrent two-phase flow in a circular pipe of radius 20 with a curved wall, D3Q19",
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


def survey_bytes_per_node(D: int, precision: str, k: int, mass_mode: int = 0):
    """Algorithmic HBM bytes per node and step of the whole step, by the
    byte model the measurement is specified with (every population of both
    distributions, P = 2Q, counted in the stream and the CG, including the
    rest direction that never streams; r nonzeros per row, n_b basis
    matrices; s_p population, s_c vector and s_v value bytes; 8 B of node
    references in deviation storage):
        stream  P s_p + ref + r (4 + n_b s_v) + P s_c
        CG      [r (4 + s_v) + 4 P s_c + s_c] + k [r (4 + s_v) + 6 P s_c + s_c]
        rest    moments, recovery and collision, a fixed figure per lattice
                and precision.
    The lumped mass drops the CG; the Chebyshev solve has no figure in that
    model (None)."""
    Q, r, nb = (9, 7, 5) if D == 2 else (19, 15, 9)
    P = 2 * Q
    sp = {"fp64": 8, "fp32": 4, "fp32_fp16": 2}[precision]
    sc = sv = 8 if precision == "fp64" else 4
    ref = 0 if precision == "fp64" else 8
    rest = {(2, 8): 1076, (2, 4): 640, (2, 2): 550, (3, 8): 2584, (3, 4): 1456}.get((D, sp))
    if rest is None or mass_mode == 2:
        return None
    stream = P * sp + ref + r * (4 + nb * sv) + P * sc
    cg = 0 if mass_mode == 1 else (r * (4 + sv) + 4 * P * sc + sc) + k * (r * (4 + sv) + 6 * P * sc + sc)
    return stream + cg + rest


def host_cpu():
    """Cores this process may run on and the host CPU model."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return dict(nproc=n, cpu_model=model)


def oracle_prefix(workload, steps: int, mass_mode: int = 0):
    """The FP64 oracle, as it stands, over `steps` steps of every instance
    (its streaming stage on all the threads the OpenMP runtime offers):
    returns the fields of each instance after the prefix and the seconds
    spent in the step loop (mesh set-up and initialisation excluded)."""
    from oracle import oracle as O
    fields, secs = [], 0.0
    for inst in workload.instances:
        o = O.Oracle(inst.mesh, workload.lattice, inst.phys, mass_mode=1 if mass_mode == 1 else 0)
        o.init(inst.rho0, inst.u0, inst.p0)
        t0 = time.perf_counter()
        o.step(steps, allow_notconv=True)
        secs += time.perf_counter() - t0
        fields.append(o.fields())
        del o
    return fields, secs, O.max_threads()


def oracle_single_thread(workload, mass_mode: int = 0):
    """One step of the largest instance with the oracle on one thread."""
    from oracle import oracle as O
    inst = max(workload.instances, key=lambda i: i.mesh["xyz"].shape[0])
    o = O.Oracle(inst.mesh, workload.lattice, inst.phys, mass_mode=1 if mass_mode == 1 else 0)
    o.set_threads(1)
    o.init(inst.rho0, inst.u0, inst.p0)
    t0 = time.perf_counter()
    o.step(1, allow_notconv=True)
    secs = time.perf_counter() - t0
    N = inst.mesh["xyz"].shape[0]
    return dict(value=N * 2 * workload.lattice / secs, unit="NPU/s", cores=1,
                sample=f"1 step of the largest instance ({N} nodes), {secs:.1f} s")


def device_prefix(ctx, workload, steps: int):
    """Fields of every instance after `steps` steps from the initial state,
    re-initialised on an already timed context (same schedule, same graph)."""
    for i, inst in enumerate(workload.instances):
        ctx.init_fields(i, inst.phys, inst.rho0, inst.u0, inst.p0)
    ctx.step(steps)
    ctx.sync(allow_notconv=True)
    return [ctx.read_fields(i) for i in range(len(workload.instances))]


def traffic_path(workload: str, precision: str, mass_mode: int, node_order: int) -> str:
    suffix = "_zorder" if node_order == 1 else ""
    return os.path.join(ROOT, "profiles", f"{workload}_traffic_{precision}_mass{mass_mode}{suffix}.json")


def measured_traffic(workload: str, precision: str, mass_mode: int, kernel: str, name: str | None,
                     node_order: int = 0):
    """HBM bytes per launch of kernel `name` (class `kernel`) from the
    committed rocprofv3 counter summary of the same workload, precision,
    mass solve and device row order (FETCH_SIZE and WRITE_SIZE scaled by
    their copy-kernel calibration), or None when no summary covers this
    configuration and kernel or the device sources changed since the
    counters were taken."""
    from paper_1608_01906_amd.profiling import device_source_hash, lookup_traffic
    path = traffic_path(workload, precision, mass_mode, node_order)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if device_source_hash() != rec["kernel_source_sha256_16"] or rec.get("node_order", 0) != node_order:
        return None
    return lookup_traffic(rec, kernel, name)


def _status(ctx):
    """'ok', or the device condition fel_sync reports (the timing stands either way)."""
    from paper_1608_01906_amd import felbm
    try:
        st = ctx.sync(allow_notconv=True)
    except felbm.FelError as e:  # non-finite state
        return str(e)
    return "ok" if st == felbm.FEL_OK else "FEL_ENOTCONV: CG residual above tolerance"


def run_gpu(w, precision, steps, warmup, prof_steps, mass_mode=0, workload="ensemble2d", node_order=0, sched=None):
    import torch
    from paper_1608_01906_amd import felbm
    N = w.n_nodes
    P = 2 * w.lattice
    ctx = felbm.from_workload(w, precision=precision, device="cuda:0", mass_mode=mass_mode, node_order=node_order,
                              **(sched or {}))
    info = ctx.layout_info()
    ctx.step(warmup)
    warm_status = _status(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    status = _status(ctx)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    if status == "ok" and warm_status != "ok":
        status = warm_status
    # event-timed pass: the same step with an event pair around every kernel
    ctx.profile(True)
    ctx.step(prof_steps)
    prof = ctx.profile_read()
    ctx.profile(False)
    s = 8 if precision == "fp64" else 4
    sp = {"fp64": 8, "fp32": 4, "fp32_fp16": 2}[precision]
    D = 2 if w.lattice == 9 else 3
    NB = 5 if D == 2 else 9
    rows = info["rows"]
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
        dom_name = solver_kernel_name(dom, precision, info["ell_width"], 2 * (w.lattice - 1), b,
                                      {2: True, 3: "wave"}.get(sg, False), sched.get("fused") == 2,
                                      info["halo_max"])
    sec_step = secs / steps
    traffic = measured_traffic(workload, precision, mass_mode, dom, dom_name, node_order)
    design_bytes = sum(v["bytes_per_launch"] * v["launches"] for v in kern.values()) / prof_steps
    spec = survey_bytes_per_node(D, precision, info["cg_iters"], mass_mode)
    res = dict(value=N * P * steps / secs, ms_per_step=sec_step * 1e3, cg_iters=info["cg_iters"],
               status=status,
               roofline=dict(bound="hbm", kernel=dom, achieved=dk["gbs"], peak=HBM_PEAK_GBS, unit="GB/s",
                             frac=round(dk["gbs"] / HBM_PEAK_GBS, 4),
                             traffic=traffic,
                             # measured HBM bytes over the same launch time: the second fraction
                             traffic_frac=None if traffic is None else
                             round(traffic / (dk["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                             bytes_per_launch=dk["bytes_per_launch"], avg_launch_us=dk["avg_us"],
                             kernel_instance=dom_name),
               step_bytes_per_node=spec,
               step_gbs=None if spec is None else round(spec * N / sec_step / 1e9, 1),
               step_frac=None if spec is None else round(spec * N / sec_step / 1e9 / HBM_PEAK_GBS, 4),
               step_design_bytes_per_node=round(design_bytes / N, 1),
               step_design_frac=round(design_bytes / sec_step / 1e9 / HBM_PEAK_GBS, 4),
               padded_rows=rows,
               kernels=kern,
               schedule=dict({k: dict(batch=v[0], staging=("direct", "lds", "lds_wave")[v[1] - 1])
                              for k, v in sched.items() if k in ("stream", "cg_init", "cg_a", "cg_b", "cheb") and k in kern},
                             reductions="fused" if sched.get("fused") == 2 else "finalize launches"),
               halo=dict(max=info["halo_max"], mean=round(info["halo_mean"], 1)),
               event_ms_per_step=round(sum(v["total_ms"] for v in kern.values()) / prof_steps, 4))
    return res, ctx


SIDE_KEYS = ("value", "ms_per_step", "status", "roofline", "step_bytes_per_node", "step_gbs", "step_frac",
             "step_design_frac", "event_ms_per_step")


def _errors(dev_fields, orc_fields, workload):
    """Per-instance errors (rho, u, p, C) against the oracle, the worst of
    each, and the unfloored relative velocity error max|du| / max|u_oracle|."""
    from tests._parity import compare_fields
    per, worst, u_rel = [], {}, 0.0
    for d, o, inst in zip(dev_fields, orc_fields, workload.instances):
        e = compare_fields(d, o, inst)
        per.append([float(f"{e[k]:.3e}") for k in ("rho", "u", "p", "C")])
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
        um = float(abs(o["u"]).max())
        if um > 0.0:
            u_rel = max(u_rel, float(abs(d["u"] - o["u"]).max()) / um)
    return dict(worst={k: float(f"{v:.3e}") for k, v in worst.items()}, u_unfloored=float(f"{u_rel:.3e}"),
                per_instance=per)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's full length)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp32_fp16"],
                    help="precision of the headline value (the FP64 plain path is measured beside it)")
    ap.add_argument("--profile-steps", type=int, default=20, help="steps of the event-timed pass")
    ap.add_argument("--oracle-steps", type=int, default=2,
                    help="steps of the prefix every instance is compared with the oracle on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 plain comparison run")
    ap.add_argument("--workload", default="ensemble2d", choices=sorted(DESCRIPTIONS),
                    help="workload (default: the 64-drop batched ensemble)")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="first copy this many MiB device-to-device (HBM counter calibration)")
    ap.add_argument("--no-chebyshev", action="store_true",
                    help="skip the run with the mass matrix solved by Chebyshev iteration")
    ap.add_argument("--no-lumped", action="store_true",
                    help="skip the run with the lumped mass matrix (the paper's own approximation)")
    ap.add_argument("--mass-mode", type=int, default=0, choices=[0, 1, 2],
                    help="mass solve of the headline run: 0 consistent (CG), 1 lumped, 2 consistent (Chebyshev)")
    ap.add_argument("--node-order", type=int, default=None, choices=[0, 1],
                    help="device row order of the headline and its FP32 side runs: 0 the workload's node order, "
                         "1 Z-order curve (default: Z-order for the large batched or tiled 2-D workloads, where "
                         "the LDS-staged kernels pay, else the workload's order); the FP64 plain run keeps the "
                         "workload's order unless this is given")
    ap.add_argument("--solver-batch", type=int, default=0, choices=[0, 1, 2, 4],
                    help="fix the solver kernels' population batch (0: tuned)")
    ap.add_argument("--lds-staging", type=int, default=0, choices=[0, 1, 2, 3],
                    help="fix the solver kernels' neighbour reads: 1 direct, 2 LDS-staged (0: tuned)")
    ap.add_argument("--fused", type=int, default=0, choices=[0, 1, 2],
                    help="fix the CG reductions: 1 finalize launches, 2 fused (0: tuned)")
    args = ap.parse_args()
    fp64_order = args.node_order if args.node_order is not None else 0
    if args.node_order is None:
        args.node_order = ZORDER_DEFAULT.get(args.workload, 0)
    sched = dict(solver_batch=args.solver_batch, lds_staging=args.lds_staging, fused_reductions=args.fused)
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(independent meshes would be spread over GPUs, a single mesh split into slabs with one-layer "
              "halos; see the design notes).", file=sys.stderr)
        sys.exit(2)

    from paper_1608_01906_amd.inputs import WORKLOADS

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
    steps = args.steps if args.steps is not None else w.steps
    inst = w.instances[0]
    N = w.n_nodes
    P = 2 * w.lattice
    print(f"bench: {args.workload}, {len(w.instances)} instances, {N} nodes, {args.precision}, {steps} steps",
          file=sys.stderr, flush=True)
    head, ctx_head = run_gpu(w, args.precision, steps, args.warmup, args.profile_steps,
                             mass_mode=args.mass_mode, workload=args.workload, node_order=args.node_order,
                             sched=sched)
    mass = {0: f"consistent, CG x{head['cg_iters']}", 1: "lumped",
            2: f"consistent, Chebyshev x{head['cg_iters']}"}[args.mass_mode]
    out = {
        "metric": "node-population updates/s + HBM roofline %, FP32-batched vs FP64 plain",
        "value": head["value"],
        "unit": "NPU/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "fp32_fp16": "f32 (f16 storage)"}[args.precision],
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS.get(args.workload, w.name), "instances": len(w.instances),
                   "nodes": N, "populations": P, "precision": args.precision,
                   "mass": mass, "dt": inst.phys.dt, "launch": "all instances in each launch, graph-replayed steps",
                   "node_order": ("workload", "z-curve")[args.node_order]},
        "roofline": head["roofline"],
    }
    for k in ("step_bytes_per_node", "step_gbs", "step_frac", "step_design_bytes_per_node", "step_design_frac",
              "padded_rows", "kernels", "schedule", "halo", "event_ms_per_step", "status"):
        out[k] = head[k]
    print(f"bench: headline {head['value']:.4g} NPU/s, {head['ms_per_step']:.3f} ms/step", file=sys.stderr,
          flush=True)
    ctx64 = None
    if not args.no_fp64 and args.precision != "fp64":
        r64, ctx64 = run_gpu(w, "fp64", steps, args.warmup, args.profile_steps, mass_mode=args.mass_mode,
                             workload=args.workload, node_order=fp64_order)
        out["fp64_plain"] = dict({k: r64[k] for k in SIDE_KEYS}, node_order=("workload", "z-curve")[fp64_order])
        out["speedup_vs_fp64_plain"] = head["value"] / r64["value"]
        print(f"bench: fp64 plain {r64['value']:.4g} NPU/s", file=sys.stderr, flush=True)
    if not args.no_chebyshev and args.mass_mode != 2:
        rch, _ = run_gpu(w, args.precision, steps, args.warmup, args.profile_steps, mass_mode=2,
                         workload=args.workload, node_order=args.node_order)
        out["chebyshev_solve"] = dict({k: rch[k] for k in SIDE_KEYS}, schedule=rch["schedule"])
    if not args.no_lumped and args.mass_mode != 1:
        rlu, _ = run_gpu(w, args.precision, steps, args.warmup, args.profile_steps, mass_mode=1,
                         workload=args.workload, node_order=args.node_order)
        out["lumped_mass"] = {k: rlu[k] for k in SIDE_KEYS}
    if not args.no_cpu_baseline:
        ns = args.oracle_steps
        dev = {args.precision: device_prefix(ctx_head, w, ns)}
        if ctx64 is not None:
            dev["fp64"] = device_prefix(ctx64, w, ns)
        print(f"bench: oracle over {ns} steps of {len(w.instances)} instances", file=sys.stderr, flush=True)
        orc_fields, secs, threads = oracle_prefix(w, ns, mass_mode=args.mass_mode)
        host = host_cpu()
        out["cpu_baseline"] = dict(
            value=N * P * ns / secs, unit="NPU/s", cores=threads, kind="oracle",
            sample=f"first {ns} steps of every instance of the same workload ({N} nodes), step loop only, "
                   f"{secs:.1f} s; plain FP64 C oracle, populations spread over {threads} OpenMP threads",
            host=host)
        print(f"bench: oracle {secs:.1f} s", file=sys.stderr, flush=True)
        out["cpu_baseline"]["single_thread"] = oracle_single_thread(w, mass_mode=args.mass_mode)
        out["error_vs_oracle"] = dict(
            steps=ns, norm="max |dev - oracle| / max(|oracle|_inf, floor), per instance as [rho, u, p, C]",
            **{prec: _errors(f, orc_fields, w) for prec, f in dev.items()})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
