"""Summarise rocprofv3 runs of bench.py into profiles/.

Input: three rocprofv3 output directories of the same bench.py command
  trace  --kernel-trace --stats   (kernel_stats.csv, kernel_trace.csv)
  fetch  --pmc FETCH_SIZE         (counter_collection.csv)
  write  --pmc WRITE_SIZE         (counter_collection.csv)
Output: profiles/<name>.md (durations, counters, calibration) and an entry
in profiles/pmc_traffic.json that bench.py reads as roofline.traffic.  With
--trace alone: the kernel statistics only.

HBM traffic per launch = FETCH_SIZE * f_fetch + WRITE_SIZE * f_write, where
f_* = (bytes a plain device copy of known size must move) / (what the same
counter reads for that copy kernel) -- the copy is bench.py's torch copy of
one state's worth of bytes.  Kernel classes follow the launch order of a
step: the x sweep (k_row), then the y and z sweeps (k_col, in that order);
"yz_sweep" is the mean over both k_col launches of a step.

Usage:
  python -m paper_1605_03958_amd.profiling --trace DIR --fetch DIR --write DIR \
      --workload 256cube_complex128 --state-bytes 268435456 --name sweeps_256cube_complex128 \
      --command "<the rocprofv3 command lines>"
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_KERNEL = "__amd_rocclr_copyBuffer"


# the device sources of the single-problem kernels
KERNEL_SOURCES = ("sscn_dev.hpp", "sscn_lines.hpp", "sscn_launch.hpp", "sscn_kernels.hip")


def source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1605_03958_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[0]


def classify(rows, match: str = ""):
    """Assign each sweep dispatch (in dispatch order) to x / y / z; sweep
    kernels whose name lacks `match` (another precision's) are left out."""
    out = []
    after_row = 0
    for r in sorted(rows, key=lambda r: int(r["Dispatch_Id"])):
        name = r["Kernel_Name"]
        if ("k_row" in name or "k_col" in name) and match not in name:
            cls = None
        elif "k_row" in name:
            cls = "x_sweep_pointwise"
            after_row = 0
        elif "k_col" in name:
            after_row += 1
            cls = "y_sweep" if after_row == 1 else "z_sweep_norm"
        elif name.startswith(COPY_KERNEL):
            cls = "copy"
        else:
            cls = None
        out.append((cls, r))
    return out


def _copy_top(acc):
    """Calibration copies: those within 10 % of the largest (a run that
    uploads states of several sizes copies each)."""
    if acc.get("copy"):
        top = max(acc["copy"])
        acc["copy"] = [v for v in acc["copy"] if v >= 0.9 * top]


def counter_means(path: str, counter: str, match: str = ""):
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    acc = defaultdict(list)
    for cls, r in classify(rows, match):
        if cls:
            acc[cls].append(float(r["Counter_Value"]))
    _copy_top(acc)
    return {k: sum(v) / len(v) for k, v in acc.items()}, {k: len(v) for k, v in acc.items()}


def trace_means(path: str, match: str = ""):
    rows = list(csv.DictReader(open(path)))
    for r in rows:
        r.setdefault("Dispatch_Id", r.get("Dispatch_Id", "0"))
    acc = defaultdict(list)
    for cls, r in classify(rows, match):
        if cls:
            acc[cls].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    _copy_top(acc)
    return {k: sum(v) / len(v) for k, v in acc.items()}


def trace_only(args) -> None:
    """Kernel statistics of a trace run alone (the persistent batch kernel,
    whose work per launch varies with the set of running instances)."""
    stats = list(csv.DictReader(open(_find(args.trace, "kernel_stats.csv"))))
    lines = [f"# rocprofv3 summary: {args.name}", "", f"Workload: `{args.workload}`.", "",
             "Command (run from the repository root on the MI355X machine):", "", "```", args.command.strip(), "```", "",
             "## Kernel statistics (--kernel-trace --stats)", "",
             "| kernel | calls | average us | min us | max us | total ms | share % |",
             "|---|---|---|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.1f} | {float(r['Percentage']):.2f} |")
    lines.append("")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"{args.name}.md"), "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def kernel_means(path: str, counter: str, match: str):
    """Mean counter value over the dispatches whose kernel name contains
    `match`, and their count."""
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if r["Counter_Name"] == counter and match in r["Kernel_Name"]]
    return (sum(vals) / len(vals) if vals else float("nan")), len(vals)


def largest_mean(path: str, counter: str, match: str) -> float:
    """Mean counter value over the dispatches of `match` within 10 % of the
    largest one."""
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if r["Counter_Name"] == counter and match in r["Kernel_Name"]]
    top = max(vals)
    big = [v for v in vals if v >= 0.9 * top]
    return sum(big) / len(big)


def batch_summary(args) -> None:
    """HBM traffic of the persistent batch kernel (k_batch_step) against its
    algorithmic bytes per launch (one step of every 2D and 3D instance of the
    all-active mix), calibrated on the torch copy of --state-bytes."""
    kib = 1024.0
    S = args.state_bytes
    # the calibration copy is the largest copy dispatch (admissions add small ones)
    cf = largest_mean(_find(args.fetch, "counter_collection.csv"), "FETCH_SIZE", COPY_KERNEL)
    cw = largest_mean(_find(args.write, "counter_collection.csv"), "WRITE_SIZE", COPY_KERNEL)
    f_fetch, f_write = S / (cf * kib), S / (cw * kib)
    stats = list(csv.DictReader(open(_find(args.trace, "kernel_stats.csv"))))
    lines = [f"# rocprofv3 summary: {args.name}", "", f"Workload: `{args.workload}`.", "",
             "Commands (run from the repository root on the MI355X machine):", "", "```", args.command.strip(), "```",
             "", "## Kernel statistics (--kernel-trace --stats)", "",
             "| kernel | calls | average us | min us | max us | share % |", "|---|---|---|---|---|---|"]
    for r in stats[:8]:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    lines += ["", "## HBM traffic per dispatch (FETCH_SIZE, WRITE_SIZE, calibrated)", "",
              "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes / launch | algorithmic bytes / launch "
              "| ratio |", "|---|---|---|---|---|---|---|"]
    for match, alg in (("k_batch_step", args.alg_bytes), ("k_batch_solo", None)):
        f, nf = kernel_means(_find(args.fetch, "counter_collection.csv"), "FETCH_SIZE", match)
        w, _ = kernel_means(_find(args.write, "counter_collection.csv"), "WRITE_SIZE", match)
        if nf == 0:
            continue
        tb = f * kib * f_fetch + w * kib * f_write
        lines.append(f"| {match} | {nf} | {f:.0f} | {w:.0f} | {tb:.4g} | "
                     f"{alg:.4g} | {tb / alg:.3f} |" if alg else
                     f"| {match} | {nf} | {f:.0f} | {w:.0f} | {tb:.4g} | (steps vary per launch) | - |")
    lines += ["", f"Calibration: the copy kernel `{COPY_KERNEL}` moves {S} bytes each way; factors "
              f"{f_fetch:.4f} (FETCH_SIZE) and {f_write:.4f} (WRITE_SIZE).", ""]
    with open(os.path.join(ROOT, "profiles", f"{args.name}.md"), "w") as fh:
        fh.write("\n".join(lines))
    print("\n".join(lines))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--state-bytes", type=int)
    ap.add_argument("--name", required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--batch", action="store_true", help="summarise the persistent batch kernel")
    ap.add_argument("--alg-bytes", type=float, default=0.0, help="algorithmic bytes per persistent launch")
    ap.add_argument("--match", default="",
                    help="only sweep kernels whose name contains this (one precision of a two-precision run)")
    args = ap.parse_args()
    if args.batch:
        batch_summary(args)
        return
    if not args.fetch or not args.write:
        trace_only(args)
        return

    stats = list(csv.DictReader(open(_find(args.trace, "kernel_stats.csv"))))
    dur = trace_means(_find(args.trace, "kernel_trace.csv"), args.match)
    fetch, nf = counter_means(_find(args.fetch, "counter_collection.csv"), "FETCH_SIZE", args.match)
    write, nw = counter_means(_find(args.write, "counter_collection.csv"), "WRITE_SIZE", args.match)
    kib = 1024.0
    S = args.state_bytes
    f_fetch = S / (fetch["copy"] * kib)
    f_write = S / (write["copy"] * kib)
    alg = 2 * S
    lines = [f"# rocprofv3 summary: {args.name}", "",
             f"Workload: `{args.workload}`; state {S} bytes; algorithmic bytes per sweep launch "
             f"(one read + one write of the state) {alg}.", "",
             "Commands (run from the repository root on the MI355X machine):", "", "```",
             args.command.strip(), "```", "",
             "## Kernel statistics (--kernel-trace --stats)", "",
             "| kernel | calls | average ns | share % |", "|---|---|---|---|"]
    for r in stats:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']):.0f} | "
                     f"{float(r['Percentage']):.2f} |")
    lines += ["", "## Per class (dispatch order within a step)", ""]
    if args.match:
        lines += [f"Sweep kernels whose name contains `{args.match}` only.", ""]
    lines += [
              "| class | mean duration us | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes / launch "
              "(calibrated) | / algorithmic | achieved GB/s (algorithmic) |", "|---|---|---|---|---|---|---|"]
    rec = {}
    # the y and z sweeps of a real-time step launch one kernel (k_col): its
    # mean over both launches is the class "yz_sweep"
    if "y_sweep" in fetch and "z_sweep_norm" in fetch:
        for d in (fetch, write, dur):
            if "y_sweep" in d and "z_sweep_norm" in d:
                d["yz_sweep"] = 0.5 * (d["y_sweep"] + d["z_sweep_norm"])
    for cls in ("x_sweep_pointwise", "y_sweep", "z_sweep_norm", "yz_sweep", "copy"):
        if cls not in fetch:
            continue
        tb = fetch[cls] * kib * f_fetch + write[cls] * kib * f_write
        d = dur.get(cls, float("nan"))
        lines.append(f"| {cls} | {d / 1e3:.1f} | {fetch[cls]:.0f} | {write[cls]:.0f} | {tb:.4g} | "
                     f"{tb / alg:.3f} | {alg / d:.0f} |")
        if cls != "copy":
            rec[cls] = {"bytes_per_launch": tb, "alg_bytes_per_launch": alg, "mean_ns": d,
                        "source_hash": source_hash()}
    lines += ["", f"Calibration: the copy kernel `{COPY_KERNEL}` moves {S} bytes each way; "
              f"FETCH_SIZE reads {fetch['copy']:.0f} KiB (factor {f_fetch:.4f}), WRITE_SIZE "
              f"{write['copy']:.0f} KiB (factor {f_write:.4f}).", "",
              f"Kernel source hash: `{source_hash()}`.", ""]
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", f"{args.name}.md"), "w") as f:
        f.write("\n".join(lines))
    jp = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    allrec = {}
    if os.path.exists(jp):
        with open(jp) as f:
            allrec = json.load(f)
    allrec[args.workload] = rec
    with open(jp, "w") as f:
        json.dump(allrec, f, indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
