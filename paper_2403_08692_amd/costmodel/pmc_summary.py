"""Summarise rocprofv3 output for one kernel: the kernel-trace statistics
(calls, average duration) and, from counter-collection runs, the per-dispatch
average of each counter.  Writes a short text summary (and optionally the
HBM-traffic JSON the benchmark reads).  With --last N only the last N
dispatches of the kernel count (a benchmark's timed steps, after the
autotuner's trial launches on a smaller sample).

  python -m paper_2403_08692_amd.costmodel.pmc_summary --kernel k_shower_flat \
      --stats DIR/..._kernel_stats.csv --trace DIR/..._kernel_trace.csv --last 10 \
      --pmc DIR1/..._counter_collection.csv ...
"""
import argparse
import csv
import glob
import json
import os
import sys


def read_csv(path):
    with open(path) as fh:
        return list(csv.DictReader(fh))


def kernel_stats(path, kernel):
    out = []
    for row in read_csv(path):
        name = row.get("Name") or row.get("KernelName") or ""
        if kernel in name:
            out.append({"name": name, "calls": int(row.get("Calls", 0)),
                        "avg_ns": float(row.get("AverageNs", 0)), "total_ns": float(row.get("TotalDurationNs", 0)),
                        "pct": float(row.get("Percentage", 0))})
    return out


def trace_durations(path, kernel):
    """[(dispatch id, ns)] of the dispatches of kernels matching `kernel`, in dispatch order."""
    out = []
    for row in read_csv(path):
        name = row.get("Kernel_Name") or row.get("Kernel-Name") or ""
        if kernel in name:
            out.append((int(row["Dispatch_Id"]), int(row["End_Timestamp"]) - int(row["Start_Timestamp"])))
    return sorted(out)


def counters(path, kernel, last=0):
    """{counter: [value per dispatch]} for dispatches of kernels matching `kernel`
    (the last `last` of them if last > 0)."""
    per = {}
    for row in read_csv(path):
        name = row.get("Kernel_Name") or row.get("Kernel-Name") or ""
        if kernel not in name:
            continue
        c = row.get("Counter_Name")
        v = float(row.get("Counter_Value", 0))
        disp = row.get("Dispatch_Id") or row.get("Correlation_Id")
        per.setdefault(c, {}).setdefault(disp, 0.0)
        per[c][disp] += v
    out = {}
    for c, d in per.items():
        keys = sorted(d, key=lambda k: int(k))
        if last > 0:
            keys = keys[-last:]
        out[c] = [d[k] for k in keys]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--stats", nargs="*", default=[])
    ap.add_argument("--trace", nargs="*", default=[], help="kernel_trace CSVs (per-dispatch durations)")
    ap.add_argument("--last", type=int, default=0, help="count only the last N dispatches of the kernel")
    ap.add_argument("--pmc", nargs="*", default=[])
    ap.add_argument("--calib", nargs="*", default=[], help="counter CSVs of the copy calibration")
    ap.add_argument("--calib-bytes", type=float, default=float(2 << 30))
    ap.add_argument("--traffic-json", default="")
    ap.add_argument("--source-hash", default="")
    args = ap.parse_args()
    lines = []
    for s in args.stats:
        for p in glob.glob(s):
            for k in kernel_stats(p, args.kernel):
                lines.append(f"kernel-trace {os.path.basename(p)}: {k['name'][:60]} calls={k['calls']} "
                             f"avg={k['avg_ns'] / 1e6:.4f} ms total={k['total_ns'] / 1e6:.3f} ms ({k['pct']:.1f}%)")
    for s in args.trace:
        for p in glob.glob(s):
            d = trace_durations(p, args.kernel)
            sel = d[-args.last:] if args.last > 0 else d
            if sel:
                ms = [ns / 1e6 for _, ns in sel]
                lines.append(f"kernel-trace {os.path.basename(p)}: last {len(sel)} of {len(d)} dispatches "
                             f"avg={sum(ms) / len(ms):.4f} ms min={min(ms):.4f} max={max(ms):.4f}")
    avg = {}
    for s in args.pmc:
        for p in glob.glob(s):
            for c, vals in counters(p, args.kernel, args.last).items():
                avg[c] = sum(vals) / len(vals)
                lines.append(f"pmc {c}: {avg[c]:.6g} per dispatch ({len(vals)} dispatches)")
    scale = {}
    for s in args.calib:
        for p in glob.glob(s):
            for c, vals in counters(p, "").items():
                if c in ("FETCH_SIZE", "WRITE_SIZE") and vals:
                    big = max(vals)
                    scale[c] = args.calib_bytes / big
                    lines.append(f"calibration {c}: copy of {args.calib_bytes:.0f} B reads {big:.6g} -> "
                                 f"{scale[c]:.4f} B per counter unit")
    traffic = None
    if "FETCH_SIZE" in avg and "WRITE_SIZE" in avg:
        fs = scale.get("FETCH_SIZE", 1024.0)
        ws = scale.get("WRITE_SIZE", 1024.0)
        traffic = avg["FETCH_SIZE"] * fs + avg["WRITE_SIZE"] * ws
        lines.append(f"HBM traffic per launch: fetch {avg['FETCH_SIZE'] * fs:.6g} B + write "
                     f"{avg['WRITE_SIZE'] * ws:.6g} B = {traffic:.6g} B")
        if args.traffic_json:
            json.dump({"kernel": args.kernel, "bytes_per_launch": traffic,
                       "fetch_bytes": avg["FETCH_SIZE"] * fs, "write_bytes": avg["WRITE_SIZE"] * ws,
                       "scale_fetch": fs, "scale_write": ws, "kernel_source_sha256": args.source_hash},
                      open(args.traffic_json, "w"), indent=1)
    print("\n".join(lines))


if __name__ == "__main__":
    sys.exit(main())
