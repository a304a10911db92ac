"""Summaries of rocprofv3 output for the profiles/ folder.

    python paper_1109_3277_amd/profile_summary.py trace  <trace_dir> --title T --cmd C [--by-grid] > out.md
    python paper_1109_3277_amd/profile_summary.py traffic <fetch_dir> <write_dir> --kernel K \
        --workload W --precision P --nodes N --bytes-per-node B --cmds C1 C2 > out.md  (+ --json out.json)

`trace` reads the kernel statistics CSV of a `rocprofv3 --kernel-trace --stats`
run and tabulates calls and average / min / max duration per kernel.

`traffic` reads the counter CSVs of two `rocprofv3 --pmc FETCH_SIZE` and
`--pmc WRITE_SIZE` runs of the same program. That program ends with one copy
by the calibration kernel (k_probe_copy16) of a known number of bytes, whose
counter readings give the factor from counter units to bytes; every kernel's
per-dispatch readings are scaled by it. The JSON record carries the hash of the
fused kernel's source, so that a reader can tell whether it still describes the
current kernel.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CALIB = "k_probe_copy16"


def _csvs(d, suffix):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {d}")
    return files


def _short(name: str) -> str:
    """Kernel name without the namespace and argument list, template arguments kept."""
    n = re.sub(r"^void\s+", "", name)
    n = n.replace("lbe::", "").replace("(anonymous namespace)::", "")
    depth, out = 0, []
    for ch in n:  # drop the parameter list after the template arguments
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        if ch == "(" and depth == 0:
            break
        out.append(ch)
    return "".join(out).strip()


def trace_by_grid(args):
    """Per (kernel, grid) statistics from the per-dispatch trace, so that one
    kernel launched on boxes of different sizes is reported per box."""
    groups = {}
    for f in _csvs(args.dir, "kernel_trace.csv"):
        for r in csv.DictReader(open(f)):
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
            groups.setdefault((_short(r["Kernel_Name"]), grid), []).append(d)
    print(f"# {args.title}\n")
    print("Command (from the repository root, on one MI355X):\n")
    print(f"    {args.cmd}\n")
    print("Per kernel and launch grid (work-items), from the per-dispatch trace.\n")
    print("| kernel | grid | calls | average (us) | min (us) | max (us) | total (ms) |")
    print("|---|---|---|---|---|---|---|")
    for (k, g), v in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        if sum(v) < args.min_total_us:
            continue
        print(f"| {k} | {g} | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} | {sum(v) / 1e3:.2f} |")


def trace(args):
    if args.by_grid:
        return trace_by_grid(args)
    rows = []
    for f in _csvs(args.dir, "kernel_stats.csv"):
        for r in csv.DictReader(open(f)):
            rows.append(r)
    print(f"# {args.title}\n")
    print("Command (from the repository root, on one MI355X):\n")
    print(f"    {args.cmd}\n")
    print("| kernel | calls | average (us) | min (us) | max (us) |")
    print("|---|---|---|---|---|")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows:
        print(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
              f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")


def _counter(d, counter):
    """{kernel: [per-dispatch values]} of one counter (KiB)."""
    out = {}
    for f in _csvs(d, "counter_collection.csv"):
        for r in csv.DictReader(open(f)):
            if r.get("Counter_Name") != counter:
                continue
            out.setdefault(_short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def traffic(args):
    fetch = _counter(args.fetch_dir, "FETCH_SIZE")
    write = _counter(args.write_dir, "WRITE_SIZE")
    cal_f, cal_w = fetch[CALIB][-1], write[CALIB][-1]
    ff = args.copy_bytes / (cal_f * 1024.0)
    wf = args.copy_bytes / (cal_w * 1024.0)
    src = os.path.join(HERE, "csrc", "lbe_fluid.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    print(f"# HBM traffic per kernel: {args.workload}, {args.precision}\n")
    print("Two counter passes (one counter each), from the repository root:\n")
    for c in args.cmds:
        print(f"    {c}")
    print(f"\nCalibration: the same runs end with {CALIB} over {args.copy_bytes / 2 ** 30:.0f} GiB "
          f"(read once, written once). FETCH_SIZE reads {cal_f:.0f} KiB for it (factor {ff:.5f}), "
          f"WRITE_SIZE {cal_w:.0f} KiB (factor {wf:.5f}). Source hash of lbe_fluid.hip: {sha}.\n")
    print("| kernel | dispatches | FETCH_SIZE KiB (mean) | WRITE_SIZE KiB (mean) | read GB | write GB |")
    print("|---|---|---|---|---|---|")
    for k in sorted(set(fetch) | set(write)):
        fv, wv = fetch.get(k, [0.0]), write.get(k, [0.0])
        mf, mw = sum(fv) / len(fv), sum(wv) / len(wv)
        print(f"| {k} | {len(fv)} | {mf:.0f} | {mw:.0f} | {mf * 1024 * ff / 1e9:.3f} | {mw * 1024 * wf / 1e9:.3f} |")
    kf, kw = fetch[args.kernel], write[args.kernel]
    # the fused kernel's dispatches of the steady steps (the median, robust to a first-step outlier)
    mf, mw = sorted(kf)[len(kf) // 2], sorted(kw)[len(kw) // 2]
    rb, wb = mf * 1024 * ff, mw * 1024 * wf
    alg = args.nodes * args.bytes_per_node
    print(f"\n{args.kernel} per launch (median dispatch): {rb / 1e9:.3f} GB read + {wb / 1e9:.3f} GB written = "
          f"{(rb + wb) / 1e9:.3f} GB, against {alg / 1e9:.3f} GB algorithmic ({args.bytes_per_node} B per node, "
          f"{args.nodes} nodes): {(rb + wb) / alg:.3f} x.")
    if args.json:
        rec = {"kernel": args.kernel, "workload": args.workload, "precision": args.precision,
               "source_sha256_16": sha, "fetch_kib_per_dispatch": mf, "write_kib_per_dispatch": mw,
               "copy_calibration": {"bytes": args.copy_bytes, "fetch_kib": cal_f, "write_kib": cal_w,
                                    "fetch_factor": ff, "write_factor": wf},
               "fetch_bytes_per_launch": int(rb), "write_bytes_per_launch": int(wb),
               "bytes_per_launch": int(rb + wb), "algorithmic_bytes_per_launch": alg, "commands": args.cmds}
        json.dump(rec, open(args.json, "w"), indent=1)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--by-grid", action="store_true", help="group the per-dispatch trace by kernel and grid")
    t.add_argument("--min-total-us", type=float, default=0.0, help="omit groups with less total time (by-grid)")
    p = sub.add_parser("traffic")
    p.add_argument("fetch_dir")
    p.add_argument("write_dir")
    p.add_argument("--kernel", required=True)
    p.add_argument("--workload", required=True)
    p.add_argument("--precision", required=True)
    p.add_argument("--nodes", type=int, required=True)
    p.add_argument("--bytes-per-node", type=int, required=True)
    p.add_argument("--copy-bytes", type=int, default=1 << 30)
    p.add_argument("--cmds", nargs=2, required=True)
    p.add_argument("--json")
    a = ap.parse_args()
    trace(a) if a.what == "trace" else traffic(a)


if __name__ == "__main__":
    sys.exit(main())
