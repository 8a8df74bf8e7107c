"""Summarise rocprofv3 output of the benchmark into a short text file under profiles/.

    python -m paper_2211_06902_amd.rocprof_summary --stats DIR --fetch DIR --write DIR \
        --copy-fetch DIR --copy-write DIR --kernel k_hop<float --out profiles/NAME.md \
        --command "..." [--bench-json FILE]

Inputs are the output directories of
  rocprofv3 --kernel-trace --stats --output-format csv ...   (per-kernel durations)
  rocprofv3 --pmc FETCH_SIZE ... / --pmc WRITE_SIZE ...         (per-dispatch KiB)
of the same benchmark command, and the same two counters on a plain device copy
of known size (bench.py --copy-calibration: 1 GiB read and written per copy),
whose ratio to the known bytes scales the counters to bytes.  The summary
records a hash of the kernel source so that readers can tell whether the
counters still describe the current kernel.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# the hop kernel's source: its kernel file and the shared stencil header
KERNEL_SOURCES = [os.path.join(HERE, "csrc", "dd_kernels.hip"), os.path.join(HERE, "csrc", "dd_stencil.h")]
GIB = float(1 << 30)


def kernel_source_hash(paths=None) -> str:
    h = hashlib.sha256()
    for path in paths or KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _one(path_dir: str, pattern: str) -> str:
    hits = sorted(glob.glob(os.path.join(path_dir, "**", pattern), recursive=True))
    if not hits:
        raise FileNotFoundError("%s not found under %s" % (pattern, path_dir))
    return hits[0]


def _counter(path_dir: str, name: str, kernel: str, skip: int = 0):
    """Per-dispatch values of counter `name` for the kernels whose name contains `kernel`, in
    dispatch order, leaving out the first `skip` of them."""
    rows = list(csv.DictReader(open(_one(path_dir, "*counter_collection.csv"))))
    hits = [r for r in rows if r["Counter_Name"] == name and kernel in r["Kernel_Name"]]
    hits.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [float(r["Counter_Value"]) for r in hits[skip:]]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--stats", required=True)
    ap.add_argument("--fetch", help="FETCH_SIZE run (omit for a timing-only summary)")
    ap.add_argument("--write")
    ap.add_argument("--copy-fetch")
    ap.add_argument("--copy-write")
    ap.add_argument("--kernel", required=True, help="substring of the kernel name")
    ap.add_argument("--alg-bytes-per-launch", type=float, help="algorithmic bytes per launch")
    ap.add_argument("--alg-flops-per-launch", type=float, help="algorithmic flops per launch (matrix-core kernels)")
    ap.add_argument("--peak", type=float, default=8000.0, help="GB/s, or TFLOP/s with --alg-flops-per-launch")
    ap.add_argument("--out", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--title", default="")
    ap.add_argument("--source", nargs="*", help="kernel source files to hash (default: the hop's)")
    ap.add_argument("--counter-skip", type=int, default=0,
                    help="average FETCH_SIZE / WRITE_SIZE leaving out the kernel's first N dispatches of each "
                         "counter run (launches of an autotuner before the measured ones)")
    ap.add_argument("--trace-skip", type=int, default=0,
                    help="average the kernel's durations from the kernel trace, leaving out its first N dispatches "
                         "(a warm-up evaluation whose first touches of fresh workspaces run slower)")
    args = ap.parse_args()

    stats = list(csv.DictReader(open(_one(args.stats, "*kernel_stats.csv"))))
    mine = [r for r in stats if args.kernel in r["Name"]]
    if not mine:
        raise SystemExit("kernel %r not in stats" % args.kernel)
    calls = sum(int(r["Calls"]) for r in mine)
    total_ns = sum(float(r["TotalDurationNs"]) for r in mine)
    avg_us = total_ns / calls / 1e3
    skip_note = ""
    if args.trace_skip:
        tr = [r for r in csv.DictReader(open(_one(args.stats, "*kernel_trace.csv"))) if args.kernel in r["Kernel_Name"]]
        tr.sort(key=lambda r: int(r["Start_Timestamp"]))
        kept = tr[args.trace_skip:]
        all_avg = avg_us
        calls = len(kept)
        avg_us = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in kept) / calls / 1e3
        skip_note = ("Average over the %d dispatches after the first %d of the trace (warm-up); over all %d: %.1f us."
                     % (calls, args.trace_skip, len(tr), all_avg))

    summary = {
        "kernel": args.kernel,
        "kernel_source_sha256_16": kernel_source_hash(args.source),
        "launches": calls,
        "avg_duration_us": avg_us,
    }
    rows = [
        "| kernel (name contains) | `%s` |" % args.kernel,
        "| launches | %d |" % calls,
        "| average duration | %.1f us |" % avg_us,
    ]
    if args.alg_bytes_per_launch:
        achieved = args.alg_bytes_per_launch / (avg_us * 1e-6) / 1e9
        summary.update(alg_bytes_per_launch=args.alg_bytes_per_launch, achieved_alg_GBs=achieved)
        rows += ["| algorithmic bytes per launch | %.4g |" % args.alg_bytes_per_launch,
                 "| achieved algorithmic bandwidth | %.0f GB/s (%.1f %% of %.0f GB/s) |"
                 % (achieved, 100 * achieved / args.peak, args.peak)]
    if args.alg_flops_per_launch:
        achieved = args.alg_flops_per_launch / (avg_us * 1e-6) / 1e12
        summary.update(alg_flops_per_launch=args.alg_flops_per_launch, achieved_TFLOPs=achieved)
        rows += ["| algorithmic flops per launch | %.4g |" % args.alg_flops_per_launch,
                 "| achieved | %.1f TFLOP/s (%.1f %% of %.0f TFLOP/s) |" % (achieved, 100 * achieved / args.peak, args.peak)]
    calib = ""
    if args.fetch:
        copy_f = _counter(args.copy_fetch, "FETCH_SIZE", "copyBuffer") or _counter(args.copy_fetch, "FETCH_SIZE", "")
        copy_w = _counter(args.copy_write, "WRITE_SIZE", "copyBuffer") or _counter(args.copy_write, "WRITE_SIZE", "")
        big_f = max(copy_f)
        big_w = max(copy_w)
        scale_f = GIB / (big_f * 1024.0)  # bytes per reported byte
        scale_w = GIB / (big_w * 1024.0)
        fv = _counter(args.fetch, "FETCH_SIZE", args.kernel, args.counter_skip)
        wv = _counter(args.write, "WRITE_SIZE", args.kernel, args.counter_skip)
        fetch_b = sum(fv) / len(fv) * 1024.0 * scale_f
        write_b = sum(wv) / len(wv) * 1024.0 * scale_w
        traffic = fetch_b + write_b
        summary.update(hbm_fetch_bytes_per_launch=fetch_b, hbm_write_bytes_per_launch=write_b,
                       hbm_traffic_bytes_per_launch=traffic, fetch_scale=scale_f, write_scale=scale_w)
        rows += ["| HBM fetch per launch (FETCH_SIZE x %.3f) | %.4g B |" % (scale_f, fetch_b),
                 "| HBM write per launch (WRITE_SIZE x %.3f) | %.4g B |" % (scale_w, write_b)]
        if args.alg_bytes_per_launch:
            summary["traffic_over_alg"] = traffic / args.alg_bytes_per_launch
            rows.append("| HBM traffic / algorithmic bytes | %.3f |" % (traffic / args.alg_bytes_per_launch))
        calib = ("Calibration: a 1 GiB device copy reads FETCH_SIZE = %.0f KiB and WRITE_SIZE = %.0f KiB per copy."
                 % (big_f, big_w))
    rows.append("| kernel source sha256[:16] | %s |" % summary["kernel_source_sha256_16"])
    if skip_note:
        summary["trace_skip"] = args.trace_skip
    if args.counter_skip:
        summary["counter_skip"] = args.counter_skip
    top = sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:12]
    lines = [
        "# %s" % (args.title or "rocprofv3 summary: " + args.kernel),
        "",
        "Command (run from the repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first):",
        "",
        "```",
        args.command,
        "```",
        "",
        "## Dominant kernel",
        "",
        "| quantity | value |",
        "|---|---|",
    ] + rows + ["", skip_note, "", calib, "",
                "## Kernel time (all kernels of the run, top 12)",
                "",
                "| kernel | calls | total ms | avg us | % |",
                "|---|---|---|---|---|"]
    for r in top:
        lines.append("| `%s` | %s | %.2f | %.1f | %.1f |" % (r["Name"][:70], r["Calls"], float(r["TotalDurationNs"]) / 1e6,
                                                       float(r["AverageNs"]) / 1e3, float(r["Percentage"])))
    lines += ["", "```json", json.dumps(summary, indent=1), "```", ""]
    with open(args.out, "w") as f:
        f.write("\n".join(lines))
    print(json.dumps(summary))


if __name__ == "__main__":
    main()
