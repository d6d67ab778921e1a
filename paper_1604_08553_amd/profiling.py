"""Summaries of rocprofv3 output for one kernel on one bench workload.

    python -m paper_1604_08553_amd.profiling --kernel sampler_kernel --workload cl1m \
        --trace DIR --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR \
        --copy-mib 512 --out profiles/ --command-file FILE

reads the CSV files rocprofv3 wrote (kernel trace + stats, FETCH_SIZE and WRITE_SIZE
counter passes over the bench, and the same two counters over a plain device copy of
known size), and writes, with NAME = the kernel's short name and the workload
(``sampler_cl1m``, ``wide_grid2000`` ...):

* ``profiles/NAME_kernel_stats.md`` -- per-kernel call counts and durations;
* ``profiles/NAME_traffic.md`` -- bytes per dispatch of the kernel leaving the L2 for the
  memory fabric (reads, FETCH_SIZE) and written (WRITE_SIZE), each counter scaled by
  (known copy bytes / what the counter read for the copy).  These count traffic below the
  L2, including reads served by the Infinity Cache, so they bound the DRAM traffic from
  above rather than measure it;
* ``profiles/NAME_traffic.json`` -- the same numbers with the SHA-256 of the kernel source
  they were taken with (bench.py reports them only while it matches);
* ``profiles/NAME_counters.md`` (with --sq-a/--sq-b/--tcc) -- wave-state and instruction
  counters and the L2 hit rate of the kernel.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCE = os.path.join(HERE, "csrc", "kad_kernels.hip")


def kernel_source_sha256() -> str:
    return hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()


def _one(pattern: str) -> str:
    files = sorted(glob.glob(pattern, recursive=True))
    if not files:
        raise FileNotFoundError(pattern)
    return files[0]


def kernel_stats(trace_dir: str):
    rows = list(csv.DictReader(open(_one(os.path.join(trace_dir, "**", "*kernel_stats.csv")))))
    return [(r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
             float(r["Percentage"])) for r in rows]


def busy_time(trace_dir: str, kernel_substr: str):
    """(dispatches, sum of durations, union of the dispatch intervals) in ns: a run's
    first main batch may run beside its pilot, so the kernel's busy time is the union."""
    path = _one(os.path.join(trace_dir, "**", "*kernel_trace.csv"))
    iv = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                for r in csv.DictReader(open(path)) if kernel_substr in r["Kernel_Name"])
    total = sum(e - b for b, e in iv)
    busy, lo, hi = 0, None, None
    for b, e in iv:
        if hi is None or b > hi:
            if hi is not None:
                busy += hi - lo
            lo, hi = b, e
        else:
            hi = max(hi, e)
    if hi is not None:
        busy += hi - lo
    return len(iv), total, busy


def counter_per_dispatch(pmc_dir: str, kernel_substr: str, counter: str):
    path = _one(os.path.join(pmc_dir, "**", "*counter_collection.csv"))
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter]
    if not vals:
        raise ValueError(f"no {counter} rows for {kernel_substr} in {path}")
    return sum(vals) / len(vals), len(vals)


WORKLOADS = {
    "cl1m": "Undirected Chung-Lu n=1,000,000, beta 2.3, mean degree 20; all-nodes, epsilon "
            "0.005, delta 0.1, seed 1.",
    "dcl4m": "Directed Chung-Lu n=4,000,000, out beta 2.5, in beta 2.1, mean degree 15; top-k "
             "k=50, epsilon 0.0002, delta 0.1, seed 1.",
    "grid2000": "2000x2000 grid with 5% of edges deleted (seed 5); hit counts of a range of "
                "main-phase sample ids, every sample with multi-limb path counts.",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", default="sampler_kernel")
    ap.add_argument("--workload", default="cl1m", choices=sorted(WORKLOADS))
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-mib", type=int, required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--sq-a", default=None, help="pass: SQ wave-cycle counters")
    ap.add_argument("--sq-b", default=None, help="pass: SQ instruction counters")
    ap.add_argument("--tcc", default=None, help="pass: TCC/TCP hit counters")
    ap.add_argument("--command-file", required=True,
                    help="text file with the exact commands that produced the inputs")
    args = ap.parse_args()
    commands = open(args.command_file).read().strip()
    os.makedirs(args.out, exist_ok=True)
    kern = args.kernel
    name = kern.replace("_kernel", "") + "_" + args.workload
    what = WORKLOADS[args.workload]

    stats = kernel_stats(args.trace)
    lines = [f"# Kernel trace: {args.workload} bench", "", what + "  Produced by:", "", "```",
             commands, "```", "",
             "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for kname, calls, tot, avg, pct in stats:
        short = kname.replace("kad::(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| {short} | {calls} | {tot / 1e6:.3f} | {avg / 1e3:.1f} | {pct:.2f} |")
    nd, tot_ns, busy_ns = busy_time(args.trace, kern)
    if nd:
        lines += ["", f"* {kern}: {nd} dispatches, mean duration {tot_ns / nd / 1e3:.1f} us; "
                  f"busy time (union of the dispatch intervals: a run's first main batch runs "
                  f"beside its pilot) {busy_ns / 1e6:.3f} ms = {busy_ns / nd / 1e3:.1f} us per "
                  f"dispatch, the figure the bench's HIP events give"]
    open(os.path.join(args.out, f"{name}_kernel_stats.md"), "w").write("\n".join(lines) + "\n")

    copy_bytes = args.copy_mib << 20
    cf, _ = counter_per_dispatch(args.copy_fetch, "copyBuffer", "FETCH_SIZE")
    cw, _ = counter_per_dispatch(args.copy_write, "copyBuffer", "WRITE_SIZE")
    fetch_factor = copy_bytes / (cf * 1024.0)
    write_factor = copy_bytes / (cw * 1024.0)
    sf, nf = counter_per_dispatch(args.fetch, kern, "FETCH_SIZE")
    sw, nw = counter_per_dispatch(args.write, kern, "WRITE_SIZE")
    fetch_b = sf * 1024.0 * fetch_factor
    write_b = sw * 1024.0 * write_factor
    rec = {"kernel": kern, "workload": args.workload,
           "kernel_source_sha256": kernel_source_sha256(),
           "fetch_kib_per_dispatch": sf, "write_kib_per_dispatch": sw, "dispatches": nf,
           "copy_fetch_factor": fetch_factor, "copy_write_factor": write_factor,
           "l2_egress_bytes_per_dispatch": fetch_b + write_b,
           "fetch_bytes_per_dispatch": fetch_b, "write_bytes_per_dispatch": write_b}
    json.dump(rec, open(os.path.join(args.out, f"{name}_traffic.json"), "w"), indent=1)
    t = [f"# Traffic below the L2 of {kern} ({args.workload} bench)", "", what, "",
         "FETCH_SIZE and WRITE_SIZE count the bytes the L2 reads from and writes to the memory "
         "fabric.  Reads that the Infinity Cache serves are included, so these figures are an "
         "upper bound on DRAM traffic, not a measurement of it.", "", "Produced by:", "", "```",
         commands, "```", "",
         f"* calibration: a plain {args.copy_mib} MiB device copy read FETCH_SIZE {cf:.0f} KiB "
         f"and WRITE_SIZE {cw:.0f} KiB, so FETCH_SIZE is scaled by {fetch_factor:.3f} and "
         f"WRITE_SIZE by {write_factor:.3f}",
         f"* {kern}, {nf} dispatches: FETCH_SIZE {sf:.0f} KiB, WRITE_SIZE {sw:.0f} KiB "
         f"per dispatch (mean)",
         f"* scaled bytes below the L2 per dispatch: read {fetch_b / 1e9:.3f} GB + write "
         f"{write_b / 1e9:.3f} GB = {(fetch_b + write_b) / 1e9:.3f} GB",
         f"* kernel source SHA-256: {rec['kernel_source_sha256']}"]
    open(os.path.join(args.out, f"{name}_traffic.md"), "w").write("\n".join(t) + "\n")
    if args.sq_a and args.sq_b and args.tcc:
        c = {}
        for d in (args.sq_a, args.sq_b, args.tcc):
            path = _one(os.path.join(d, "**", "*counter_collection.csv"))
            acc = {}
            for r in csv.DictReader(open(path)):
                if kern in r["Kernel_Name"]:
                    acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
            c.update({k: sum(v) / len(v) for k, v in acc.items()})
        wave = c.get("SQ_WAVE_CYCLES", 0.0) or 1.0
        hit, miss = c.get("TCC_HIT_sum", 0.0), c.get("TCC_MISS_sum", 0.0)
        lines = [f"# Counters of {kern} ({args.workload} bench), mean per dispatch", "", what, "",
                 "Produced by:", "", "```", commands, "```", "",
                 "| counter | value |", "|---|---|"]
        lines += [f"| {k} | {v:.4g} |" for k, v in sorted(c.items())]
        lines += ["", f"* waves waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES): {c.get('SQ_WAIT_ANY', 0) / wave:.3f}",
                  f"* waves issuing (SQ_ACTIVE_INST_ANY / SQ_WAVE_CYCLES): {c.get('SQ_ACTIVE_INST_ANY', 0) / wave:.3f}",
                  f"* L2 hit rate (TCC_HIT / (TCC_HIT + TCC_MISS)): {hit / max(hit + miss, 1.0):.3f}",
                  f"* LDS bank conflicts per LDS instruction: "
                  f"{c.get('SQ_LDS_BANK_CONFLICT', 0) / max(c.get('SQ_INSTS_LDS', 1), 1):.3f}",
                  f"* kernel source SHA-256: {rec['kernel_source_sha256']}"]
        open(os.path.join(args.out, f"{name}_counters.md"), "w").write("\n".join(lines) + "\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
