"""Summaries of rocprofv3 output for the profiles/ folder.

traffic   HBM bytes per launch of each kernel class from two counter runs
          (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by
          what the same counter reads for a device copy of known size made
          in the same run (bench.py --copy-probe MiB);
stats     kernel-time statistics (rocprofv3 --kernel-trace --stats) per
          kernel class.

    python -m paper_1608_01906_amd.profiling traffic FETCH.csv WRITE.csv \\
        --copy-mib 256 --workload channel2d --precision fp32 --mass-mode 0 \\
        --command "..." --command "..." --out profiles/NAME.json
    python -m paper_1608_01906_amd.profiling stats STATS.csv --title ... \\
        --command "..." --out profiles/NAME.md

A traffic summary records a hash of the device sources; bench.py ignores
it (reports traffic null) once the kernels have changed.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
DEVICE_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("felbm_device.h", "felbm_kernels.hip", "felbm_solver.hip")]
COPY_KERNEL = "__amd_rocclr_copyBuffer"


def device_source_hash() -> str:
    h = hashlib.sha256()
    for path in DEVICE_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def kernel_class(name: str) -> str | None:
    """Kernel class (as in fel_profile_read) of a demangled kernel name:
    LDS-staged and fused forms count as their kernel."""
    m = re.search(r"fel::(k_[a-z_0-9]+?)(?:_lds|_fused)?(?:<|\()", name)
    if not m:
        return None
    k = m.group(1)[2:]
    if k.startswith("cheb"):
        return "cheb"
    for suffix in ("_plain", "_dev"):
        if k.endswith(suffix):
            k = k[: -len(suffix)]
    return k


def _per_dispatch(path: str, counter: str):
    """{class: {kernel name: [values per dispatch]}} and the copy kernel's values."""
    per = defaultdict(lambda: defaultdict(list))
    copy = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            v = float(r["Counter_Value"])
            if COPY_KERNEL in r["Kernel_Name"]:
                copy.append(v)
                continue
            k = kernel_class(r["Kernel_Name"])
            if k:
                per[k][r["Kernel_Name"]].append(v)
    return per, copy


def short_name(name: str) -> str:
    """Kernel name without 'void ' and the argument list."""
    return re.sub(r"\(.*", "", name).replace("void ", "").strip()


def staged_halo_rounds(halo_max: int, tile: int = 256) -> int:
    """Halo rounds of the staged instantiation a layout runs: its stage row
    holds the tile and the largest halo rounded up to 64; 2 rounds when the
    halo part fits in 2 tiles, else 4."""
    sw = (tile + halo_max + 63) // 64 * 64
    return 2 if sw - tile <= 2 * tile else 4


def solver_kernel_name(cls: str, precision: str, W: int, NP: int, batch: int, staged,
                       fused: bool = False, halo_max: int = 0) -> str:
    """Short name of the solver kernel a schedule launches (cheb: the
    iterate kernel, which runs all but the first of each solve).  staged:
    False direct, True a stage per tile (the kernel carries the halo rounds
    of the layout, largest halo halo_max), "wave" a stage per wavefront
    (halo rounds 0)."""
    T = "double" if precision == "fp64" else "float"
    if fused and cls in ("cg_init", "cg_a", "cg_b"):
        return f"fel::k_{cls}_fused<{T}, {W}, {NP}, {batch}>"
    if staged == "wave":
        return f"fel::k_{cls}_lds<{T}, {W}, {NP}, {batch}, 0>"
    if staged:
        return f"fel::k_{cls}_lds<{T}, {W}, {NP}, {batch}, {staged_halo_rounds(halo_max)}>"
    return f"fel::k_{cls}<{T}, {W}, {NP}, {batch}>"


def traffic(fetch_csv: str, write_csv: str, copy_mib: float, workload: str, precision: str, mass_mode: int,
            commands: list[str], node_order: int = 0) -> dict:
    """Per kernel class and instantiation: dispatches, mean counters and
    calibrated bytes per dispatch.  The autotuner's timing launches of the
    candidate schedules are dispatches of the same kernels on the same
    layout, so every candidate is covered."""
    fetch, fcopy = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write, wcopy = _per_dispatch(write_csv, "WRITE_SIZE")
    if not fcopy or not wcopy:
        raise SystemExit("no copy-kernel dispatch in the counter runs (run bench.py with --copy-probe)")
    kib = copy_mib * 1024.0
    # the copy reads and writes copy_mib each; use its largest dispatch
    ff, wf = kib / max(fcopy), kib / max(wcopy)
    out = dict(workload=workload, precision=precision, mass_mode=mass_mode, node_order=node_order,
               kernel_source_sha256_16=device_source_hash(), fetch_factor=round(ff, 4), write_factor=round(wf, 4),
               calibration=f"{copy_mib:g} MiB device-to-device copy ({COPY_KERNEL}): FETCH_SIZE {max(fcopy):.1f} "
                           f"KiB, WRITE_SIZE {max(wcopy):.1f} KiB per dispatch for {kib:.0f} KiB moved each way",
               commands=commands, kernels={})
    for k in sorted(set(fetch) & set(write)):
        inst = {}
        for name, fv in fetch[k].items():
            wv = write[k].get(name)
            if not wv:
                continue
            fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
            inst[short_name(name)] = dict(dispatches=len(fv), fetch_kib=round(fk, 1), write_kib=round(wk, 1),
                                          traffic_bytes=int(round((fk * ff + wk * wf) * 1024)))
        out["kernels"][k] = inst
    return out


def lookup_traffic(rec: dict, cls: str, name: str | None = None):
    """Bytes per dispatch of kernel `name` of class `cls` in a traffic
    record (of the class's only / most dispatched kernel when name is None),
    or None."""
    inst = rec.get("kernels", {}).get(cls)
    if not inst:
        return None
    if name is None:
        name = max(inst, key=lambda n: inst[n]["dispatches"])
    k = inst.get(name)
    return k["traffic_bytes"] if k else None


def stats(stats_csv: str, title: str, commands: list[str], bench_json: str | None = None) -> str:
    rows = defaultdict(lambda: [0, 0.0, []])
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            k = kernel_class(r["Name"])
            if not k:
                continue
            calls = int(r["Calls"])
            tot = float(r["TotalDurationNs"])
            rows[k][0] += calls
            rows[k][1] += tot
            rows[k][2].append((tot / max(calls, 1) / 1e3, calls, r["Name"]))
    lines = [f"# {title}", "", "Command(s):", ""]
    lines += [f"    {c}" for c in commands]
    lines += ["", "Per kernel class (all dispatches of the run, tuning candidates included):", "",
              "| class | calls | total ms | avg us |", "|---|---|---|---|"]
    for k, (calls, tot, _) in sorted(rows.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"| {k} | {calls} | {tot / 1e6:.3f} | {tot / max(calls, 1) / 1e3:.3f} |")
    lines += ["", "Per kernel instantiation (the schedule the tuner kept has the most calls):", "",
              "| class | avg us | calls | kernel |", "|---|---|---|---|"]
    for k in sorted(rows, key=lambda k: -rows[k][1]):
        for avg, calls, name in sorted(rows[k][2], key=lambda t: -t[1]):
            lines.append(f"| {k} | {avg:.3f} | {calls} | `{short_name(name)}` |")
    if bench_json:
        with open(bench_json) as f:
            rec = json.loads(f.read().strip().splitlines()[-1])
        rf = rec["roofline"]
        lines += ["", "bench.py line of the same command run without the profiler (HIP events around each",
                  "launch of its event-timed pass; the per-launch averages above should agree):", "",
                  f"- value {rec['value']:.4g} {rec['unit']}, {rec['ms_per_step']:.4f} ms/step (graph replay)",
                  f"- dominant kernel {rf['kernel']} (`{rf.get('kernel_instance')}`): {rf['avg_launch_us']} us per "
                  f"launch, {rf['bytes_per_launch']} algorithmic bytes, {rf['achieved']} GB/s = {rf['frac']} of "
                  f"{rf['peak']} GB/s",
                  "", "| class | event avg us | launches | algorithmic GB/s |", "|---|---|---|---|"]
        for k, v in sorted(rec["kernels"].items(), key=lambda kv: -kv[1]["total_ms"]):
            lines.append(f"| {k} | {v['avg_us']} | {v['launches']} | {v['gbs']} |")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--copy-mib", type=float, required=True)
    t.add_argument("--workload", required=True)
    t.add_argument("--precision", required=True)
    t.add_argument("--mass-mode", type=int, required=True)
    t.add_argument("--node-order", type=int, default=0, help="device row order of the counted run")
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--out", required=True)
    s = sub.add_parser("stats")
    s.add_argument("stats_csv")
    s.add_argument("--title", required=True)
    s.add_argument("--command", action="append", default=[])
    s.add_argument("--bench-json", help="bench.py output of the same command run without the profiler")
    s.add_argument("--out", required=True)
    a = ap.parse_args()
    if a.cmd == "traffic":
        rec = traffic(a.fetch_csv, a.write_csv, a.copy_mib, a.workload, a.precision, a.mass_mode, a.command,
                      a.node_order)
        with open(a.out, "w") as f:
            json.dump(rec, f, indent=1)
    else:
        with open(a.out, "w") as f:
            f.write(stats(a.stats_csv, a.title, a.command, a.bench_json))
    print(a.out)


if __name__ == "__main__":
    main()
