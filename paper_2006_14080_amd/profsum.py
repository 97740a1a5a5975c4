"""Condense rocprofv3 CSV output into the short text summaries kept in profiles/.

    python -m paper_2006_14080_amd.profsum stats <run_kernel_stats.csv> --cmd "<command>" [--top N]
    python -m paper_2006_14080_amd.profsum pmc <run_counter_collection.csv> --cmd "<command>"
    python -m paper_2006_14080_amd.profsum traffic <fetch.csv> <write.csv> --cmd "<command>" [--json out.json --key fp32]
    python -m paper_2006_14080_amd.profsum vecbw <run_kernel_stats.csv> <run log> --cmd "<command>" [--copy-bytes B]
                                           [--fetch <FETCH_SIZE csv> --write <WRITE_SIZE csv>]
    python -m paper_2006_14080_amd.profsum busy <run_kernel_trace.csv> --cmd "<command>"
    python -m paper_2006_14080_amd.profsum grid <run_kernel_trace.csv> --cmd "<command>"
    python -m paper_2006_14080_amd.profsum clock <counter_collection.csv> --cmd "<command>"

``vecbw`` turns the durations of the solver's memory-bound kernels into
achieved bandwidth from their algorithmic bytes per pixel (listed in
VEC_BYTES), against the 8 TB/s HBM peak.  The pixel count (all slices), coil
count and adjoint partial images per slice come from the run's own output
(the line ``npix=N coils=C planes=P`` that the profile driver and the batch
benchmark print, the plane count from the library's mri_adjoint_split), and
a figure above the peak is an error: it means the byte count is wrong.

``grid`` lists the NUDFT kernels of a run per (kernel, grid size), so runs
that launch one kernel at several shapes keep them apart.

``stats`` lists per-kernel call counts and durations; ``pmc`` averages every
counter per kernel over its dispatches (FETCH_SIZE / WRITE_SIZE are KiB per
dispatch as rocprofv3 reports them).
"""
import argparse
import collections
import csv
import sys


_POLICIES = {"PolF32": "PolF32", "PolSplitIDF16bLb0": "PolBF16", "PolSplitIDF16_Lb1": "PolF16"}


def _unmangle(name: str) -> str:
    """Readable names for the templated NUDFT kernels that the profiler leaves
    mangled (their template arguments include 16-bit float types)."""
    import re
    m = re.match(r"_ZN3mri12_GLOBAL__N_1\d+(nudft_(?:fwd|adj8?))INS0_\d+(\w+?)E+(?:Li(\d)E)?", name)
    if m:
        nt = f", {m.group(3)}" if m.group(3) else ""
        return f"{m.group(1)}<{_POLICIES.get(m.group(2), m.group(2))}{nt}>(mri::NudftTable)"
    m = re.match(r"_ZN3mri12_GLOBAL__N_1\d+(\w+?)ENS_10NudftTableE", name)
    if m:
        return f"{m.group(1)}(mri::NudftTable)"
    return name


def short(name: str) -> str:
    name = _unmangle(name)
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
        # Derived: matrix-core busy fraction (four SIMDs per CU) and VALU
        # instructions per MFMA instruction.
        if "SQ_VALU_MFMA_BUSY_CYCLES" in counters and counters.get("SQ_BUSY_CU_CYCLES"):
            busy = counters["SQ_VALU_MFMA_BUSY_CYCLES"] / (4.0 * counters["SQ_BUSY_CU_CYCLES"])
            extra = f"  -> matrix cores busy {busy:.1%} of CU-busy cycles"
            if counters.get("SQ_INSTS_MFMA"):
                extra += f", {counters.get('SQ_INSTS_VALU', 0.0) / counters['SQ_INSTS_MFMA']:.1f} VALU per MFMA"
            out.append(extra)
        # Derived: LDS use.  GRBM_GUI_ACTIVE is reported summed over the XCDs,
        # so the GPU's cycles in the dispatch are its value / XCDS; LDS counters
        # are summed over all CUs.
        if "SQ_LDS_IDX_ACTIVE" in counters and counters.get("GRBM_GUI_ACTIVE"):
            cyc = counters["GRBM_GUI_ACTIVE"] / n / XCDS
            cu_cyc = cyc * CUS
            rd = counters.get("SQ_INSTS_LDS_LOAD_BANDWIDTH", 0.0) / n * 64
            wr = counters.get("SQ_INSTS_LDS_STORE_BANDWIDTH", 0.0) / n * 64
            out.append(f"  -> LDS busy {counters['SQ_LDS_IDX_ACTIVE'] / n / cu_cyc:.1%} of cycles, "
                       f"bank-conflict stalls {counters.get('SQ_LDS_BANK_CONFLICT', 0.0) / n / cu_cyc:.1%}, "
                       f"ds_read {rd / 1e6:.0f} MB + ds_write {wr / 1e6:.0f} MB per dispatch "
                       f"= {(rd + wr) / cu_cyc:.1f} B/clk per CU")
    return out


XCDS, CUS = 8, 256      # MI355X


# Algorithmic bytes per pixel (complex64 = 8 B) of each memory-bound kernel:
# every array element the kernel must read or write once.
VEC_BYTES = {
    "k_mu": lambda c, p: 8 + 16 + 16,                  # rho, eta -> mu
    "k_rhs": lambda c, p: 8 + 16 + 16 + 8,             # F^H d, mu, eta -> b
    "k_adj_finish<0>": lambda c, p: 8 * p + 8,                # partial images -> F^H d
    "k_adj_finish<1>": lambda c, p: 8 * p + 8 + 8 + 3 * 8,    # partials, x, b -> r, p, x (CG start)
    "k_adj_finish<2>": lambda c, p: 8 * p + 8 + 8,            # partials, d -> A d (CG step)
    "k_cg_update": lambda c, p: 4 * 8 + 2 * 8,         # x, r, d, A d -> x, r
    "k_cg_dir": lambda c, p: 2 * 8 + 8,                # r, d -> d
    "k_dual": lambda c, p: 8 + 16 + 16 + 8 + 16 + 8,   # x, mu, eta, rho -> eta, rho
    "k_coil_weight": lambda c, p: 8 + 8 * c,           # x -> s (.) x per coil (the profiled workloads share
                                                       # one map set over all slices: read once, not per pixel)
}
HBM_PEAK = 8.0e12


def run_sizes(log_path):
    """(npix, coils, planes) from the last ``npix=N coils=C planes=P`` line of a run's output."""
    import re
    found = None
    for line in open(log_path, errors="replace"):
        m = re.search(r"npix=(\d+) coils=(\d+) planes=(\d+)", line)
        if m:
            found = tuple(int(v) for v in m.groups())
    if found is None:
        raise SystemExit(f"{log_path}: no 'npix=N coils=C planes=P' line (run the profile driver or the batch bench)")
    return found


# HBM bytes from the counters: FETCH_SIZE x 2 (it counts each 128-byte read
# request as 64 bytes) + WRITE_SIZE x 1.  Measured on the multi-GB sweep, where
# the memory-bound kernels' reads and writes are known exactly: k_cg_update
# (32 B/px read, 16 written), k_dual (48, 24), k_adj_finish<2> (16, 8) read
# exactly twice their raw FETCH_SIZE and write exactly their raw WRITE_SIZE.
# (A device copy cannot calibrate this at these sizes: the 256 MB Infinity
# Cache serves part of its reads and absorbs part of its writes.)
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0


def vecbw(path, npix, coils, planes, copy_bytes=None, fetch_csv=None, write_csv=None):
    """Per memory-bound kernel: algorithmic bytes per pixel, achieved GB/s and
    fraction of the HBM peak; with FETCH_SIZE / WRITE_SIZE counter runs of the
    same command, also the HBM bytes per pixel the counters measured."""
    rows = list(csv.DictReader(open(path)))
    meas = {}
    if fetch_csv and write_csv:
        f = _per_kernel(fetch_csv, "FETCH_SIZE")
        w = _per_kernel(write_csv, "WRITE_SIZE")
        cf, cw = FETCH_SCALE, WRITE_SCALE
        for k in f:
            if k in w and k != COPY_KERNEL:
                meas[k.split("(")[0].replace("void ", "").strip()] = (f[k] * 1024.0 * cf + w[k] * 1024.0 * cw) / npix
    head = f"{'kernel':16s} {'calls':>6s} {'avg_us':>9s} {'bytes/px':>9s} {'GB/s':>8s} {'of 8 TB/s':>9s}"
    out = [head + (f" {'HBM B/px (counters)':>20s}" if meas else "")]
    if copy_bytes:
        # a device copy of copy_bytes read + copy_bytes written, in the same run
        for r in rows:
            if short(r["Name"]).startswith(COPY_KERNEL) and float(r["AverageNs"]) > 1e5:
                gbs = 2 * copy_bytes / (float(r["AverageNs"]) * 1e-9) / 1e9
                out.append(f"{'(device copy)':16s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                           f"{'-':>9s} {gbs:8.1f} {gbs * 1e9 / HBM_PEAK:9.1%}")
    for r in rows:
        k = short(r["Name"]).split("(")[0].replace("void ", "").strip()
        if k not in VEC_BYTES:
            continue
        b = VEC_BYTES[k](coils, planes)
        us = float(r["AverageNs"]) / 1e3
        gbs = b * npix / (us * 1e-6) / 1e9
        if gbs * 1e9 > HBM_PEAK:
            raise SystemExit(f"{k}: {gbs:.0f} GB/s exceeds the HBM peak; its byte count "
                             f"({b} B/px, {planes} planes) does not match the run")
        line = f"{k:16s} {int(r['Calls']):6d} {us:9.2f} {b:9d} {gbs:8.1f} {gbs * 1e9 / HBM_PEAK:9.1%}"
        if meas:
            line += f" {meas.get(k, float('nan')):20.1f}"
        out.append(line)
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


KERNEL_SOURCES = ["nudft.hip", "phase.h", "device.h", "internal.h"]


def _code_only(text: str) -> str:
    """C++ source without comments and whitespace (string literals in these
    kernel sources hold no comment markers)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return re.sub(r"\s+", "", text)


def kernel_fingerprint() -> str:
    """sha256 over the code of the NUDFT kernel sources, comments and
    whitespace excluded (traffic is void once the code changes)."""
    import hashlib
    import os
    h = hashlib.sha256()
    base = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for n in KERNEL_SOURCES:
        with open(os.path.join(base, n)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()


SIMDS = CUS * 4
PEAK_CLOCK_GHZ = 2.4     # GRBM_GUI_ACTIVE is summed over the XCDS dies


def clock(path):
    """Per NUDFT dispatch: duration, shader clock (GRBM_GUI_ACTIVE per die over
    the duration) and matrix-core busy cycles as a fraction of the SIMD cycles
    at the peak clock and at the measured one; dispatches grouped into
    quartiles of their duration."""
    rows = list(csv.DictReader(open(path)))
    d = collections.defaultdict(dict)
    for r in rows:
        k = short(r["Kernel_Name"])
        if "nudft_" not in k:
            continue
        e = d[k].setdefault(r["Dispatch_Id"], {"us": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3})
        e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    out = []
    for k, disp in d.items():
        xs = sorted(disp.values(), key=lambda e: e["us"])
        out.append(f"{k}: {len(xs)} dispatches")
        out.append("  duration quartile   avg_us   clock_GHz   MFMA busy / SIMD cycles at 2.4 GHz   at the measured clock")
        q = max(1, len(xs) // 4)
        for i in range(4):
            part = xs[i * q:(i + 1) * q] if i < 3 else xs[3 * q:]
            if not part:
                continue
            us = sum(e["us"] for e in part) / len(part)
            ghz = sum(e["GRBM_GUI_ACTIVE"] / XCDS / (e["us"] * 1e3) for e in part) / len(part)
            f_peak = sum(e["SQ_VALU_MFMA_BUSY_CYCLES"] / (SIMDS * PEAK_CLOCK_GHZ * e["us"] * 1e3) for e in part) / len(part)
            f_clk = sum(e["SQ_VALU_MFMA_BUSY_CYCLES"] / (SIMDS * e["GRBM_GUI_ACTIVE"] / XCDS) for e in part) / len(part)
            out.append(f"  Q{i + 1:<17d} {us:8.1f}   {ghz:9.3f}   {f_peak:33.3f}   {f_clk:21.3f}")
    return out


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


def busy(trace_csv, top):
    """GPU busy fraction between the first and last NUDFT kernel of a kernel
    trace (union of kernel intervals), and time per kernel in that window."""
    rows = list(csv.DictReader(open(trace_csv)))
    ev = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short(r["Kernel_Name"]).split("(")[0])
                for r in rows)
    nud = [x for x in ev if x[2].startswith("nudft")]
    t0, t1 = nud[0][0], nud[-1][1]
    win = [x for x in ev if x[0] >= t0 and x[1] <= t1]
    covered, cur_s, cur_e = 0, None, None
    for s, e, _ in win:
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                covered += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    covered += cur_e - cur_s
    agg = collections.defaultdict(lambda: [0, 0])
    for s, e, k in win:
        agg[k][0] += 1
        agg[k][1] += e - s
    out = [f"window {(t1 - t0) / 1e9:.2f} s, GPU busy {covered / 1e9:.2f} s ({covered / (t1 - t0):.1%})",
           f"{'kernel':40s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>10s}"]
    for k, (c, t) in sorted(agg.items(), key=lambda x: -x[1][1])[:top]:
        out.append(f"{k:40s} {c:6d} {t / 1e6:10.1f} {t / c / 1e3:10.1f}")
    return out


def grid(trace_csv):
    """Calls and average duration per (NUDFT kernel, grid size)."""
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        k = short(r["Kernel_Name"])
        if not k.startswith("nudft"):
            continue
        agg[(k, int(r.get("Grid_Size") or r["Grid_Size_X"]))].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = [f"{'kernel':44s} {'grid (threads)':>15s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s}"]
    for (k, g), d in sorted(agg.items(), key=lambda x: (x[0][0], -x[0][1])):
        out.append(f"{k:44s} {g:15d} {len(d):6d} {sum(d) / len(d):10.2f} {min(d):10.2f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("mode", choices=["stats", "pmc", "traffic", "vecbw", "busy", "grid", "clock"])
    ap.add_argument("csv")
    ap.add_argument("csv2", nargs="?")
    ap.add_argument("--cmd", required=True)
    ap.add_argument("--top", type=int, default=14)
    ap.add_argument("--json")
    ap.add_argument("--key")
    ap.add_argument("--copy-bytes", type=int, help="vecbw: size of the reference device copy in the run")
    ap.add_argument("--fetch", help="vecbw: FETCH_SIZE counter csv of the same command")
    ap.add_argument("--write", help="vecbw: WRITE_SIZE counter csv of the same command")
    a = ap.parse_args()
    if a.mode == "vecbw":
        npix, coils, planes = run_sizes(a.csv2)
        print("# solver memory-bound kernels: achieved bandwidth from algorithmic bytes")
        print(f"# command: {a.cmd}")
        print(f"# pixels (all slices) = {npix}, coils = {coils}, adjoint partial images per slice = {planes} "
              "(as printed by the run)")
        if a.fetch:
            print(f"# HBM bytes from FETCH_SIZE / WRITE_SIZE runs of the same command: FETCH_SIZE x {FETCH_SCALE:g} "
                  f"+ WRITE_SIZE x {WRITE_SCALE:g} (KiB per dispatch)")
        for line in vecbw(a.csv, npix, coils, planes, a.copy_bytes, a.fetch, a.write):
            print(line)
        return 0
    if a.mode == "busy":
        print("# GPU busy time of a run from its rocprofv3 kernel trace")
        print(f"# command: {a.cmd}")
        for line in busy(a.csv, a.top):
            print(line)
        return 0
    if a.mode == "traffic":
        t = traffic(a.csv, a.csv2)
        t["command"] = a.cmd
        t["kernel_sources_sha256"] = kernel_fingerprint()
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
    if a.mode == "clock":
        print("# NUDFT dispatches of a run: duration, shader clock and matrix-core busy fraction")
        print(f"# command: {a.cmd}")
        print(f"# clock = GRBM_GUI_ACTIVE / {XCDS} dies / duration; busy fraction = SQ_VALU_MFMA_BUSY_CYCLES over "
              f"{SIMDS} SIMDs x cycles")
        for line in clock(a.csv):
            print(line)
        return 0
    if a.mode == "grid":
        print("# NUDFT kernels per launch shape from a rocprofv3 kernel trace")
        print(f"# command: {a.cmd}")
        for line in grid(a.csv):
            print(line)
        return 0
    print(f"# rocprofv3 summary ({a.mode})")
    print(f"# command: {a.cmd}")
    for line in (stats(a.csv, a.top) if a.mode == "stats" else pmc(a.csv)):
        print(line)


if __name__ == "__main__":
    sys.exit(main())
