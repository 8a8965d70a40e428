"""Summaries of rocprofv3 output for the step kernel.

Reads the CSV files of a kernel-trace (--kernel-trace --stats) run and of
two counter runs (--pmc FETCH_SIZE, --pmc WRITE_SIZE) of
paper_2009_05264_amd/profile_run.py, and writes

* profiles/<name>.md: kernel statistics and the scaled memory traffic per
  launch, with the commands that produced the CSV files;
* an entry in profiles/traffic_step_kernel.json (read by bench.py): HBM
  bytes per step-kernel launch for that workload, valid for the kernel
  source whose hash it records.

Counter scaling: profile_run.py ends with three copies of a known byte count
through the library's copy kernel; bytes read (written) by one copy divided
by the mean FETCH_SIZE (WRITE_SIZE) reading of those dispatches, in bytes,
is the factor applied to the step kernel's readings.

    python3 paper_2009_05264_amd/prof_summary.py --name step_kernel_channel_8192x1024 \
        --workload 8192x1024 --storage F32_DEV --kt DIR --fetch DIR --write DIR --copy-mib 1024
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import re
import json
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# the step kernel, the host code that shapes its tiles, and the header with
# the store-policy threshold
KERNEL_SRC = [os.path.join(HERE, "csrc", f) for f in ("lbm_kernels.hip", "lbm_tiles.cpp", "lbm_internal.h")]
TRAFFIC = os.path.join(ROOT, "profiles", "traffic_step_kernel.json")


def kernel_sha() -> str:
    return hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SRC)).hexdigest()[:16]


def _one(dirname: str, suffix: str) -> str:
    hits = glob.glob(os.path.join(dirname, f"*{suffix}"))
    if len(hits) != 1:
        raise FileNotFoundError(f"expected one *{suffix} in {dirname}, found {hits}")
    return hits[0]


def kernel_stats(dirname: str):
    rows = list(csv.DictReader(open(_one(dirname, "kernel_stats.csv"))))
    return [(r["Name"], int(r["Calls"]), float(r["AverageNs"]), float(r["MinNs"]), float(r["MaxNs"]),
             float(r["Percentage"])) for r in rows]


def counter(dirname: str, name: str):
    """Mean counter value (KiB) per dispatch of the step kernel and of the copy kernel."""
    step, copy = [], []
    for r in csv.DictReader(open(_one(dirname, "counter_collection.csv"))):
        if r["Counter_Name"] != name:
            continue
        k = r["Kernel_Name"]
        if re.search(r"step_kernel<\d+, 0(, (true|false))?>", k):  # storage, MODE_STEP[, store policy]
            step.append(float(r["Counter_Value"]))
        elif "copy_kernel" in k:
            copy.append(float(r["Counter_Value"]))
    if not step or not copy:
        raise ValueError(f"{dirname}: no {name} readings for the step or copy kernel")
    return statistics.mean(step), statistics.mean(copy), len(step), len(copy)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--name", required=True)
    ap.add_argument("--workload", required=True, help="e.g. 1600x200")
    ap.add_argument("--storage", default="F32_DEV")
    ap.add_argument("--kt", required=True, help="kernel-trace output directory")
    ap.add_argument("--fetch", required=True, help="FETCH_SIZE output directory")
    ap.add_argument("--write", required=True, help="WRITE_SIZE output directory")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--kt-cmd", default="")
    ap.add_argument("--pmc-cmd", default="")
    ap.add_argument("--alg-bytes", type=float, required=True, help="algorithmic bytes per launch")
    args = ap.parse_args()

    ks = kernel_stats(args.kt)
    f_step, f_copy, nf, nfc = counter(args.fetch, "FETCH_SIZE")
    w_step, w_copy, nw, nwc = counter(args.write, "WRITE_SIZE")
    copy_bytes = args.copy_mib << 20
    f_scale = copy_bytes / (f_copy * 1024.0)
    w_scale = copy_bytes / (w_copy * 1024.0)
    rd = f_step * 1024.0 * f_scale
    wr = w_step * 1024.0 * w_scale
    step = [k for k in ks if re.search(r"step_kernel<\d+, 0(, (true|false))?>", k[0])]
    avg_ns = step[0][2] if step else float("nan")

    lines = [f"# step_kernel, workload {args.workload}, storage {args.storage}", "",
             f"kernel and tiling source sha256[:16]: `{kernel_sha()}`", ""]
    if args.kt_cmd:
        lines += ["Kernel trace command:", "", "```", args.kt_cmd, "```", ""]
    lines += ["| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for name, calls, avg, mn, mx, pct in ks[:6]:
        short = name.replace("void ", "").replace("(anonymous namespace)::", "").split("(")[0]
        lines.append(f"| `{short}` | {calls} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | {pct:.2f} |")
    lines += [""]
    if args.pmc_cmd:
        lines += ["Counter commands (one pass per counter, C = FETCH_SIZE, then WRITE_SIZE):", "", "```",
                  args.pmc_cmd, "```", ""]
    lines += [
        "| counter | step kernel (KiB/dispatch, mean) | copy kernel (KiB/dispatch) | scale | step kernel bytes |",
        "|---|---|---|---|---|",
        f"| FETCH_SIZE | {f_step:.1f} (n={nf}) | {f_copy:.1f} (n={nfc}) | {f_scale:.4f} | {rd / 1e6:.1f} MB |",
        f"| WRITE_SIZE | {w_step:.1f} (n={nw}) | {w_copy:.1f} (n={nwc}) | {w_scale:.4f} | {wr / 1e6:.1f} MB |",
        "",
        f"Copy calibration: {args.copy_mib} MiB read and written per copy dispatch.",
        f"Memory traffic per launch (L2 misses and write-backs, FETCH_SIZE + WRITE_SIZE; served by HBM or by "
        f"the Infinity Cache): {(rd + wr) / 1e6:.1f} MB; algorithmic bytes per launch "
        f"{args.alg_bytes / 1e6:.1f} MB (ratio {(rd + wr) / args.alg_bytes:.3f}).",
    ]
    if step:
        lines.append(f"Kernel-trace mean duration {avg_ns / 1e3:.2f} us: algorithmic "
                     f"{args.alg_bytes / avg_ns:.1f} GB/s, measured memory traffic {(rd + wr) / avg_ns:.1f} GB/s.")
    out_md = os.path.join(ROOT, "profiles", args.name + ".md")
    os.makedirs(os.path.dirname(out_md), exist_ok=True)
    open(out_md, "w").write("\n".join(lines) + "\n")

    tr = json.load(open(TRAFFIC)) if os.path.exists(TRAFFIC) else {}
    if tr.get("kernel_sha") != kernel_sha():
        tr = {"kernel_sha": kernel_sha(), "entries": {}}
    tr["entries"][f"{args.workload}/{args.storage}"] = {
        "bytes_per_launch": round(rd + wr), "read_bytes": round(rd), "write_bytes": round(wr),
        "fetch_scale": f_scale, "write_scale": w_scale, "kernel_trace_avg_us": avg_ns / 1e3,
        "summary": os.path.relpath(out_md, ROOT)}
    json.dump(tr, open(TRAFFIC, "w"), indent=1)
    print(open(out_md).read())


if __name__ == "__main__":
    main()
