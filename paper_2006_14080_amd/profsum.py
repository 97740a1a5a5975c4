"""Condense rocprofv3 CSV output into the short text summaries kept in profiles/.

    python -m paper_2006_14080_amd.profsum stats <run_kernel_stats.csv> --cmd "<command>" [--top N]
    python -m paper_2006_14080_amd.profsum pmc <run_counter_collection.csv> --cmd "<command>"

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "pmc"])
    ap.add_argument("csv")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--top", type=int, default=14)
    a = ap.parse_args()
    print(f"# rocprofv3 summary ({a.mode})")
    print(f"# command: {a.cmd}")
    for line in (stats(a.csv, a.top) if a.mode == "stats" else pmc(a.csv)):
        print(line)


if __name__ == "__main__":
    sys.exit(main())
