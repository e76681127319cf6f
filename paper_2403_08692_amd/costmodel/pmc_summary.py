"""Summarise rocprofv3 output for one kernel: the kernel-trace statistics
(calls, average duration) and, from counter-collection runs, the per-dispatch
average of each counter.  Writes a short text summary (and optionally the
HBM-traffic JSON the benchmark reads).

  python -m paper_2403_08692_amd.costmodel.pmc_summary --kernel k_shower_plain \
      --stats DIR/..._kernel_stats.csv --pmc DIR1/..._counter_collection.csv ...
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


def counters(path, kernel):
    """{counter: [value per dispatch]} for dispatches of kernels matching `kernel`."""
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
    return {c: list(d.values()) for c, d in per.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--stats", nargs="*", default=[])
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
    avg = {}
    for s in args.pmc:
        for p in glob.glob(s):
            for c, vals in counters(p, args.kernel).items():
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
