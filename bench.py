"""Benchmark: ADMM-TV reconstruction throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|bf16x3|fp16x3]
                    [--workload admm256|slices384|table1_1024x512|serve]

One step = one full admm_solve of the 256x256, 8-coil, 64x512-sample radial
problem (30 ADMM iterations x 5 CG steps: 1 + 2*30*6 = 361 NUDFT calls),
inputs resident in HBM.  value = ADMM iterations per second over the K timed
steps.  Also reported:

* roofline -- the dominant NUDFT kernel: algorithmic flop per launch
  (8 * nk * nx * ny * nc) over its average launch time, measured with HIP
  events on the stream it runs on, against the MI355X dense FP32 MFMA peak
  (BF16 / FP16 peak for the split forms, where each product costs three);
  the adjoint is timed as the solve launches it (phase tables prepared once);
* cpu_baseline -- the FP64 NumPy oracle timed on the host on a bounded sample
  (one ADMM iteration with 5 CG steps of the same problem);
* image_nrmse_vs_oracle -- the timed solve's image against the oracle's own
  30 x 5 reconstruction of the same data (stored under tests/golden), and
  image_nrmse_vs_phantom against the ground-truth phantom;
* forms_at_equal_nrmse -- FP32 at 30 x 5 beside each split form (bf16x3,
  fp16x3) run for as many ADMM iterations as it takes to reach FP32's image
  NRMSE against the phantom to three significant figures, with the seconds
  per reconstruction of each;
* latency_p50_s / latency_p99_s -- reconstruction latency over a short
  Poisson trace (24 mixed-shape requests at 0.3 req/s, below the FP32
  saturation knee) replayed against the continuous-batching server.

Other workloads (one JSON line each):

* slices384 -- 32 slices of 384x384, 16 coils, 128x768 samples in one batched
  solve; one step = one ADMM iteration (5 CG) over the whole batch;
* table1_1024x512 -- the large-image case of Sec. VI (1024x512 grid, 12
  coils, 101x1024 samples per coil) with the Table I parameters: relative
  tolerance 1e-4 over at most 5 ADMM iterations, CG absolute tolerance 1e-6
  over at most 20 steps, both evaluated on the device; one step = one whole
  reconstruction, reported in seconds;
* serve -- a Poisson stream of mixed-shape requests (128/256/384 pixels,
  4-32 coils, 32-128 spokes x 2N, 30 ADMM x 5 CG) replayed in wall-clock time
  against the request server; reports p50/p99 latency and recons/s.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2516.6, "fp16x3": 2516.6}   # MI355X dense MFMA peaks
DTYPE = {"fp32": "f32", "bf16x3": "bf16x3", "fp16x3": "f16x3", "nufft": "f32"}
# Oracle data and 30 x 5 reconstruction of the 256x256 problem
# (written by tests/golden/make_admm256_golden.py).
GOLDEN_ADMM256 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden", "admm256_oracle.npz")
# Oracle data and 2 x 2 reconstructions of slices 0 and 31 of the 32-slice
# 384x384 batch (tests/golden/make_slices384_golden.py).
GOLDEN_SLICES384 = os.path.join(ROOT, "tests", "golden", "slices384_oracle.npz")
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp32", "bf16x3", "fp16x3", "nufft"], default="fp32",
                    help="NUDFT arithmetic form, or nufft: F by the NUFFT operator (width 6, oversampling 2)")
    ap.add_argument("--workload", choices=["admm256", "slices384", "table1_1024x512", "serve"],
                    default="admm256")
    ap.add_argument("--requests", type=int, default=24, help="serve: requests in the replayed stream")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: mean arrival rate (req/s)")
    ap.add_argument("--slots", type=int, default=8, help="serve: concurrent slots")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: device pool (GiB)")
    ap.add_argument("--kernel-launches", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve-latency", action="store_true",
                    help="admm256: skip the served trace behind latency_p50_s / latency_p99_s")
    ap.add_argument("--no-equal-nrmse", action="store_true",
                    help="admm256: skip the comparison of the precision forms at equal image NRMSE")
    ap.add_argument("--latency-requests", type=int, default=24)
    ap.add_argument("--latency-rate", type=float, default=0.3,
                    help="admm256: arrival rate of the latency trace (req/s), under the FP32 knee (~0.45)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "nudft_traffic_admm256.json"),
                    help="JSON with measured HBM bytes per launch of the NUDFT kernels (optional)")
    return ap.parse_args()


def cpu_baseline(wl, p):
    """Oracle timed on one ADMM iteration (5 CG steps) of the same problem."""
    from oracle import admm as oadmm
    from oracle import nudft as onudft
    blas = "unknown"
    try:
        from threadpoolctl import threadpool_info
        info = threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] or [1])
        blas = ", ".join(sorted({f"{i.get('internal_api')} {i.get('version')}" for i in info
                                 if i.get("user_api") == "blas"})) or blas
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next(line.split(":", 1)[1].strip() for line in f if line.startswith("model name"))
    except Exception:  # pragma: no cover
        pass
    data = (onudft.forward(p.truth[0], p.smaps, p.traj) + p.noise[0]).astype(np.complex64)
    t0 = time.perf_counter()
    oadmm.admm(data, p.smaps, p.traj, wl.lam, wl.beta, 1, wl.cg_iters)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "ADMM iters/s", "cores": int(threads), "kind": "oracle",
            "host": {"cpu_model": cpu_model, "cpu_count": os.cpu_count(), "blas": blas},
            "sample": f"1 ADMM iteration x {wl.cg_iters} CG ({1 + 2 * (1 + wl.cg_iters)} NUDFT calls incl. F^H d) of "
                      f"{wl.name}, FP64 NumPy, {dt:.1f} s"}


def bench_slices(args):
    """32-slice 384x384 batch: ADMM iterations per second of the whole batch."""
    import torch
    from paper_2006_14080_amd import mri, synth

    prec = mri.PRECISIONS[args.precision]
    wl = synth.SLICES384
    p = synth.make_problem(wl)
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    sm, tr, truth = g(p.smaps), g(p.traj), g(p.truth)
    data = mri.nudft_forward(truth, sm, tr, precision=mri.FP32)
    data += g(p.noise.astype(np.complex64))
    torch.cuda.synchronize()
    shape = mri.shape_of((wl.batch, wl.ny, wl.nx), sm, tr)
    # sizes for the memory-bound kernels' bandwidth summary (profsum vecbw)
    print(f"npix={wl.batch * wl.nx * wl.ny} coils={wl.nc} planes={mri.adjoint_split(shape)['planes']}",
          file=sys.stderr, flush=True)
    steps, warm = max(1, args.steps), args.warmup
    # admm_iters = warmup + timed iterations; F^H d and the init run before the timed region
    stream = torch.cuda.current_stream()
    out = torch.empty((wl.batch, wl.ny, wl.nx), dtype=torch.complex64, device=dev)
    timings = {}
    for n_it in (warm, warm + steps):
        solver = mri.AdmmSolver(shape, mri.AdmmParams(wl.lam, wl.beta, n_it, wl.cg_iters, precision=prec), device=dev)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        solver.solve(sm, tr, data, out=out)
        b.record(stream)
        torch.cuda.synchronize()
        timings[n_it] = a.elapsed_time(b)
        st = solver.stats()
        assert all(s["status"] == 0 and s["admm_iters"] == n_it for s in st), st[:2]
        del solver
    ms_step = (timings[warm + steps] - timings[warm]) / steps
    flop_iter = wl.nudft_flop * 2 * (1 + wl.cg_iters)
    # Image error: the same batch with slices 0 and 31 on the data stored with
    # the oracle's reconstructions of them (tests/golden, 2 ADMM x 2 CG).
    img_err = None
    if os.path.exists(GOLDEN_SLICES384):
        gold = np.load(GOLDEN_SLICES384)
        d2 = data.clone()
        for i, b in enumerate(gold["slices"]):
            d2[int(b)] = g(gold["data"][i])
        solver = mri.AdmmSolver(shape, mri.AdmmParams(wl.lam, wl.beta, int(gold["admm_iters"]),
                                                      int(gold["cg_iters"]), precision=prec), device=dev)
        solver.solve(sm, tr, d2, out=out)
        torch.cuda.synchronize()
        img_err = {"admm_iters": int(gold["admm_iters"]), "cg_iters": int(gold["cg_iters"])}
        for i, b in enumerate(gold["slices"]):
            got = out[int(b)].cpu().numpy().astype(np.complex128)
            ref = gold["images"][i].astype(np.complex128)
            img_err[f"slice{int(b)}"] = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        del solver, d2
    rec = {
        "metric": "ADMM iters/s over a 32-slice 384x384 batch (16 coils, 128x768 samples, 5 CG per iteration)",
        "value": 1e3 / ms_step, "unit": "ADMM iters/s (whole batch)", "n_gpus": 1, "steps": steps,
        "warmup": warm, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[args.precision],
        "data": "synthetic (32 seeded ellipse phantoms, shared Gaussian coil maps and golden-angle trajectory)",
        "config": {"workload": wl.name, "batch": wl.batch, "nx": wl.nx, "ny": wl.ny, "coils": wl.nc,
                   "spokes": wl.n_spokes, "readout": wl.n_readout, "cg_iters": wl.cg_iters,
                   "precision": args.precision,
                   "note": "one step = one full ADMM iteration of all 32 slices; the difference of two solves "
                           "with warmup and warmup+steps iterations isolates the per-iteration time"},
        "fp32_equiv_tflops": flop_iter / ms_step / 1e9,
        "slice_iters_per_s": wl.batch * 1e3 / ms_step,
        "image_nrmse_vs_oracle": img_err,
    }
    print(json.dumps(rec), flush=True)


def bench_table1_large(args):
    """1024x512 / 12-coil reconstruction with the Table I stopping rules: seconds per solve."""
    import torch
    from paper_2006_14080_amd import mri, synth

    prec = mri.PRECISIONS[args.precision]
    wl = synth.TABLE1_1024x512
    p = synth.make_problem(wl)
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    sm, tr, truth = g(p.smaps), g(p.traj), g(p.truth)
    data = mri.nudft_forward(truth, sm, tr, precision=mri.FP32)
    data += g(p.noise.astype(np.complex64))
    torch.cuda.synchronize()
    params = mri.AdmmParams(wl.lam, wl.beta, wl.admm_iters, wl.cg_iters, rtol=wl.rtol, atol=wl.atol,
                            precision=prec)
    solver = mri.AdmmSolver(mri.shape_of((1, wl.ny, wl.nx), sm, tr), params, device=dev)
    out = torch.empty((1, wl.ny, wl.nx), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        solver.solve(sm, tr, data, out=out)
    torch.cuda.synchronize()
    times, stats = [], []
    for i in range(max(1, args.steps)):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        solver.solve(sm, tr, data, out=out)
        b.record(stream)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
        stats.append(solver.stats()[0])
        print(f"[table1_1024x512] solve {i + 1}: {times[-1]:.3f} s", file=sys.stderr, flush=True)
    st = stats[-1]
    if st["status"] != 0:
        raise RuntimeError(f"solve failed: {st}")
    calls = 1 + 2 * (st["admm_iters"] + st["cg_steps"])
    s_solve = float(np.mean(times))
    got = out[0].cpu().numpy().astype(np.complex128)
    truth0 = p.truth[0].astype(np.complex128)
    rec = {
        "metric": "seconds per 1024x512 reconstruction (12 coils, 101x1024 radial samples, Table I stopping rules)",
        "value": s_solve, "unit": "s", "n_gpus": 1, "steps": len(times), "warmup": args.warmup,
        "ms_per_step": 1e3 * s_solve, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[args.precision],
        "data": "synthetic (seeded ellipse phantom, Gaussian coil maps, golden-angle radial trajectory, "
                "k-space data F(phantom) formed on the GPU plus complex Gaussian noise 1e-3)",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "coils": wl.nc, "spokes": wl.n_spokes,
                   "readout": wl.n_readout, "admm_max": wl.admm_iters, "cg_max": wl.cg_iters,
                   "lambda": wl.lam, "beta": wl.beta, "rtol": wl.rtol, "atol": wl.atol,
                   "precision": args.precision},
        "admm_iters_run": int(st["admm_iters"]), "cg_steps_run": int(st["cg_steps"]),
        "nudft_calls": calls,
        "fp32_equiv_tflops": wl.nudft_flop * calls / s_solve / 1e12,
        "solve_s_all": times,
        "image_nrmse_vs_phantom": float(np.linalg.norm(got - truth0) / np.linalg.norm(truth0)),
    }
    print(json.dumps(rec), flush=True)


def run_served_trace(prec, n_requests, rate, slots, budget_gb, progress_s=30.0):
    """Replay a Poisson stream of mixed-shape requests against the request
    server in wall-clock time; returns (replay result, total NUDFT flop,
    arrival times)."""
    import torch
    from paper_2006_14080_amd import mri, serve, synth

    reqs = synth.request_stream(n_requests, rate=rate)
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    payloads, flop = [], 0.0
    for i, r in enumerate(reqs):   # k-space data: F(phantom) on the GPU plus seeded noise, staged on the host
        if i % 25 == 0:
            print(f"[serve] preparing request {i}/{len(reqs)}", file=sys.stderr, flush=True)
        p = synth.make_problem(r.wl)
        d = mri.nudft_forward(g(p.truth), g(p.smaps), g(p.traj), precision=mri.FP32)[0].cpu().numpy()
        d = (d + p.noise[0]).astype(np.complex64)
        payloads.append(dict(smaps=p.smaps, traj=p.traj, data=d,
                             params=mri.AdmmParams(r.wl.lam, r.wl.beta, r.wl.admm_iters, r.wl.cg_iters)))
        flop += r.wl.nudft_flop * r.wl.nudft_calls
    torch.cuda.synchronize()
    arrivals = [r.arrival for r in reqs]
    with serve.Server(int(budget_gb * (1 << 30)), max_slots=slots, precision=prec) as srv:
        res = serve.replay(srv, arrivals, payloads, progress_s=progress_s)
    return res, flop, arrivals


def bench_serve(args):
    """Mixed-shape request stream through the continuous-batching server."""
    from paper_2006_14080_amd import mri

    prec = mri.PRECISIONS[args.precision]
    res, flop, arrivals = run_served_trace(prec, args.requests, args.rate, args.slots, args.budget_gb)
    rec = {
        "metric": "served ADMM-TV reconstructions: p50/p99 latency and recons/s",
        "value": res["recons_per_s"], "unit": "recons/s", "n_gpus": 1, "steps": args.requests, "warmup": 0,
        "ms_per_step": 1e3 * res["wall_s"] / args.requests, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[args.precision],
        "data": "synthetic (seeded phantoms, Gaussian coil maps, golden-angle radial trajectories)",
        "config": {"workload": f"serve_poisson{args.rate:g}_n{args.requests}", "rate_req_s": args.rate,
                   "requests": args.requests, "slots": args.slots, "budget_gib": args.budget_gb,
                   "sizes": [128, 256, 384], "coils": [4, 32], "spokes": [32, 128], "readout": "2N",
                   "admm_iters": 30, "cg_iters": 5, "precision": args.precision},
        "latency_p50_s": res["p50_s"], "latency_p99_s": res["p99_s"],
        "latency_mean_s": float(np.mean(res["latency_s"])), "wall_s": res["wall_s"],
        "offered_load_tflop_per_s": flop / (max(arrivals) - min(arrivals) + 1e-9) / 1e12,
        "served_fp32_equiv_tflops": flop / res["wall_s"] / 1e12,
        "server": {k: int(v) for k, v in res["info"].items()},
    }
    print(json.dumps(rec), flush=True)


def sig3(v: float) -> str:
    return f"{v:.3g}"


def forms_at_equal_nrmse(wl, sm, tr, data, truth0, max_iters=90):
    """The precision forms compared at equal image quality: FP32 runs the
    workload's 30 x 5; each split form runs 30, 31, ... ADMM iterations (5 CG
    each) until its image NRMSE against the phantom, at three significant
    figures, is no larger than FP32's (or max_iters is reached); `matched_3sf`
    says whether the two agree to three figures there.  Seconds per
    reconstruction are HIP-event times of one whole solve."""
    import torch
    from paper_2006_14080_amd import mri

    stream = torch.cuda.current_stream()
    shape = mri.shape_of((1, wl.ny, wl.nx), sm, tr)
    out = torch.empty((1, wl.ny, wl.nx), dtype=torch.complex64, device=data.device)

    def run(prec, n):
        solver = mri.AdmmSolver(shape, mri.AdmmParams(wl.lam, wl.beta, n, wl.cg_iters, precision=prec),
                                device=data.device)
        solver.solve(sm, tr, data, out=out)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        solver.solve(sm, tr, data, out=out)
        b.record(stream)
        torch.cuda.synchronize()
        got = out[0].cpu().numpy().astype(np.complex128)
        return float(np.linalg.norm(got - truth0) / np.linalg.norm(truth0)), a.elapsed_time(b) / 1e3

    e32, t32 = run(mri.FP32, wl.admm_iters)
    res = {"fp32": {"admm_iters": wl.admm_iters, "nrmse_vs_phantom": e32, "s_per_recon": t32}}
    for name in ("bf16x3", "fp16x3"):
        prec = mri.PRECISIONS[name]
        reached = False
        for n in range(wl.admm_iters, max_iters + 1):
            e, t = run(prec, n)
            if float(sig3(e)) <= float(sig3(e32)):
                reached = True
                break
        res[name] = {"admm_iters": n, "nrmse_vs_phantom": e, "s_per_recon": t, "reached": reached,
                     "matched_3sf": sig3(e) == sig3(e32), "speedup_vs_fp32": t32 / t}
        print(f"[equal-nrmse] {name}: {n} ADMM iterations, NRMSE vs phantom {e:.5f} (fp32 {e32:.5f}), "
              f"{t:.3f} s vs {t32:.3f} s", file=sys.stderr, flush=True)
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU k-space split (its design is documented, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "slices384":
        return bench_slices(args)
    if args.workload == "table1_1024x512":
        return bench_table1_large(args)
    if args.workload == "serve":
        return bench_serve(args)
    import torch
    from paper_2006_14080_amd import mri, synth

    prec = mri.PRECISIONS[args.precision]
    wl = synth.ADMM256
    p = synth.make_problem(wl)
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    sm, tr, truth = g(p.smaps), g(p.traj), g(p.truth)
    # Synthetic k-space data F(phantom) + seeded complex noise: the copy stored
    # beside the oracle's own 30 x 5 reconstruction of this problem when it is
    # there (so the final image can be compared with it), else formed on the GPU.
    golden = None
    if os.path.exists(GOLDEN_ADMM256):
        golden = np.load(GOLDEN_ADMM256)
        data = g(golden["data"][None])
    else:
        data = mri.nudft_forward(truth, sm, tr, precision=mri.FP32)
        data += g(p.noise.astype(np.complex64))
    torch.cuda.synchronize()

    params = mri.AdmmParams(wl.lam, wl.beta, wl.admm_iters, wl.cg_iters, precision=prec)
    shape = mri.shape_of((1, wl.ny, wl.nx), sm, tr)
    solver = mri.AdmmSolver(shape, params, device=dev)
    out = torch.empty((1, wl.ny, wl.nx), dtype=torch.complex64, device=dev)

    for _ in range(args.warmup):
        solver.solve(sm, tr, data, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        solver.solve(sm, tr, data, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    st = solver.stats()[0]
    if st["status"] != 0 or st["admm_iters"] != wl.admm_iters:
        raise RuntimeError(f"solve did not run to completion: {st}")
    iters_per_s = wl.admm_iters * args.steps / (ms_total / 1e3)
    nrmse = None
    got = out[0].cpu().numpy().astype(np.complex128)
    if golden is not None:
        ref = golden["image"].astype(np.complex128)
        nrmse = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
    truth0 = p.truth[0].astype(np.complex128)
    nrmse_truth = float(np.linalg.norm(got - truth0) / np.linalg.norm(truth0))

    # Per-kernel timing of the two NUDFT operators at the solve's launch
    # configuration (same kernels, tables and stream as inside admm_solve).
    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(n):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    dtmp = torch.empty_like(data)
    img = out.clone()
    if prec == mri.NUFFT:
        nplan = mri.NufftPlan(sm, tr, wl.ny, wl.nx)
        fwd_ms = timed(lambda: nplan.forward(img, out=dtmp), args.kernel_launches)
        adj_ms = timed(lambda: nplan.adjoint(data, out=img), args.kernel_launches)
    else:
        fwd_ms = timed(lambda: mri.nudft_forward(img, sm, tr, precision=prec, out=dtmp), args.kernel_launches)
        # The adjoint as the solve applies it: phase tables built once for the
        # trajectory, then the adjoint kernel and its fixed-order reduction.
        adj = mri.AdjointPlan(sm, tr, wl.ny, wl.nx, precision=prec)
        adj_ms = timed(lambda: adj(data, out=img), args.kernel_launches)
    flop = wl.nudft_flop
    dom_name, dom_ms = ("nudft_forward", fwd_ms) if fwd_ms >= adj_ms else ("nudft_adjoint", adj_ms)
    achieved = flop / (dom_ms / 1e3) / 1e12
    if prec in (mri.BF16X3, mri.FP16X3):
        achieved_pipe = achieved * 3.0      # three 16-bit products per real product
    else:
        achieved_pipe = achieved
    peak = PEAK_TFLOPS.get(args.precision)
    # HBM bytes per launch from FETCH_SIZE / WRITE_SIZE (copy-calibrated), valid
    # only while the kernel sources match the ones the counters were taken on.
    traffic = None
    if os.path.exists(args.traffic):
        try:
            from paper_2006_14080_amd.profsum import kernel_fingerprint
            with open(args.traffic) as f:
                rec_t = json.load(f).get(args.precision, {})
            if rec_t.get("kernel_sources_sha256") == kernel_fingerprint():
                traffic = rec_t.get(dom_name, {}).get("bytes")
        except Exception:
            traffic = None

    rec = {
        "metric": "ADMM iters/s (256x256, 8 coils, 64x512 radial samples, 30 ADMM x 5 CG)",
        "value": iters_per_s,
        "unit": "ADMM iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic (seeded ellipse phantom, Gaussian coil maps, golden-angle radial trajectory, "
                "complex Gaussian noise 1e-3)",
        "config": {"workload": wl.name, "nx": wl.nx, "ny": wl.ny, "coils": wl.nc, "spokes": wl.n_spokes,
                   "readout": wl.n_readout, "admm_iters": wl.admm_iters, "cg_iters": wl.cg_iters,
                   "lambda": wl.lam, "beta": wl.beta, "precision": args.precision,
                   "nudft_calls_per_step": wl.nudft_calls},
        "roofline": ({"bound": "mfma", "kernel": dom_name, "achieved": achieved_pipe, "peak": peak,
                      "unit": "TFLOP/s", "frac": achieved_pipe / peak, "traffic": traffic,
                      "algorithmic_tflop_per_launch": flop / 1e12,
                      "avg_launch_ms": dom_ms} if peak else None),
        "kernels_ms": {"nudft_forward": fwd_ms, "nudft_adjoint": adj_ms,
                       "fp32_equiv_tflops": {"nudft_forward": flop / fwd_ms / 1e9,
                                             "nudft_adjoint": flop / adj_ms / 1e9}},
        "wall_s_timed": wall,
        "image_nrmse_vs_oracle": nrmse,
        "image_nrmse_vs_phantom": nrmse_truth,
    }
    if prec == mri.NUFFT:
        rec["note"] = ("F by the NUFFT operator (Kaiser-Bessel width 6, oversampling 2, FP32): its kernels are "
                       "grid, FFT and gather passes, not a matrix product, so no MFMA roofline; kernels_ms holds "
                       "its forward and adjoint times and fp32_equiv_tflops the dense product's flop over them")
    if not args.no_equal_nrmse and prec != mri.NUFFT:
        rec["forms_at_equal_nrmse"] = forms_at_equal_nrmse(wl, sm, tr, data, truth0)
    if not args.no_serve_latency and prec != mri.NUFFT:
        # The latency half of the metric: a short Poisson trace of mixed-shape
        # requests (128/256/384 px, 4-32 coils, 32-128 spokes, 30 x 5 each) at
        # an arrival rate under the form's saturation knee, replayed in wall-clock
        # time against the continuous-batching server.
        res, sflop, arr = run_served_trace(prec, args.latency_requests, args.latency_rate, 8, 64.0)
        rec["latency_p50_s"] = res["p50_s"]
        rec["latency_p99_s"] = res["p99_s"]
        rec["latency_trace"] = {"workload": f"serve_poisson{args.latency_rate:g}_n{args.latency_requests}",
                                "rate_req_s": args.latency_rate, "requests": args.latency_requests,
                                "recons_per_s": res["recons_per_s"], "wall_s": res["wall_s"],
                                "latency_mean_s": float(np.mean(res["latency_s"])),
                                "served_fp32_equiv_tflops": sflop / res["wall_s"] / 1e12}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(wl, p)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
