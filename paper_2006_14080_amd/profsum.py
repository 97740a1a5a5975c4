"""Condense rocprofv3 CSV output into the short text summaries kept in profiles/.

    python -m paper_2006_14080_amd.profsum stats <run_kernel_stats.csv> --cmd "<command>" [--top N]
    python -m paper_2006_14080_amd.profsum pmc <run_counter_collection.csv> --cmd "<command>"
    python -m paper_2006_14080_amd.profsum traffic <fetch.csv> <write.csv> --cmd "<command>" [--json out.json --key fp32]

``stats`` lists per-kernel call counts and durations; ``pmc`` averages every
counter per kernel over its dispatches (FETCH_SIZE / WRITE_SIZE are KiB per
dispatch as rocprofv3 reports them).
"""
import argparse
import collections
import csv
import sys


def short(name: str) -> str:
    name = name.replace("mri::(anonymous namespace)::", "").replace("(anonymous namespace)::", "")
    return name.replace("void ", "")[:90]


def stats(path, top):
    rows = list(csv.DictReader(open(path)))
    out = [f"{'kernel':90s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}"]
    for r in rows[:top]:
        out.append(f"{short(r['Name']):90s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}")
    return out


def pmc(path):
    rows = list(csv.DictReader(open(path)))
    val = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    dur = collections.defaultdict(dict)
    for r in rows:
        k = short(r["Kernel_Name"])
        val[k][r["Counter_Name"]] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
        dur[k][r["Dispatch_Id"]] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    out = []
    for k, counters in val.items():
        n = len(disp[k])
        avg_us = sum(dur[k].values()) / max(1, len(dur[k]))
        items = ", ".join(f"{c}={v / n:.6g}" for c, v in sorted(counters.items()))
        out.append(f"{k}: dispatches={n} avg_us={avg_us:.2f} {items}")
    return out


COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 256 * 1024 * 1024      # the driver's calibration copy reads and writes 256 MiB


def _per_kernel(path, counter):
    rows = list(csv.DictReader(open(path)))
    val = collections.defaultdict(float)
    disp = collections.defaultdict(set)
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        k = short(r["Kernel_Name"])
        val[k] += float(r["Counter_Value"])
        disp[k].add(r["Dispatch_Id"])
    return {k: v / len(disp[k]) for k, v in val.items()}   # KiB per dispatch


def traffic(fetch_csv, write_csv):
    """HBM bytes per dispatch, each counter scaled by its reading for the copy."""
    f = _per_kernel(fetch_csv, "FETCH_SIZE")
    w = _per_kernel(write_csv, "WRITE_SIZE")
    cf = COPY_BYTES / (f[COPY_KERNEL] * 1024.0)
    cw = COPY_BYTES / (w[COPY_KERNEL] * 1024.0)
    out = {"calibration": {"fetch_scale": cf, "write_scale": cw,
                           "copy_fetch_kib": f[COPY_KERNEL], "copy_write_kib": w[COPY_KERNEL]}}
    for k in f:
        if k == COPY_KERNEL or k not in w:
            continue
        name = "nudft_forward" if k.startswith("nudft_fwd") else "nudft_adjoint" if k.startswith("nudft_adj") else k
        out[name] = {"fetch_bytes": f[k] * 1024.0 * cf, "write_bytes": w[k] * 1024.0 * cw,
                     "bytes": f[k] * 1024.0 * cf + w[k] * 1024.0 * cw,
                     "raw_fetch_kib": f[k], "raw_write_kib": w[k]}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "pmc", "traffic"])
    ap.add_argument("csv")
    ap.add_argument("csv2", nargs="?")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--top", type=int, default=14)
    ap.add_argument("--json")
    ap.add_argument("--key")
    a = ap.parse_args()
    if a.mode == "traffic":
        t = traffic(a.csv, a.csv2)
        t["command"] = a.cmd
        if a.json:
            import json
            import os
            d = json.load(open(a.json)) if os.path.exists(a.json) else {}
            d[a.key] = t
            with open(a.json, "w") as fh:
                json.dump(d, fh, indent=1, sort_keys=True)
        for k, v in t.items():
            print(k, v)
        return 0
    print(f"# rocprofv3 summary ({a.mode})")
    print(f"# command: {a.cmd}")
    for line in (stats(a.csv, a.top) if a.mode == "stats" else pmc(a.csv)):
        print(line)


if __name__ == "__main__":
    sys.exit(main())
