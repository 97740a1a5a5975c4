"""Fixed workloads for profiler runs (rocprofv3 --pmc / --stats).

    python -m paper_2006_14080_amd.profile_driver [fp32|bf16x3|fp16x3] [repeats]
    python -m paper_2006_14080_amd.profile_driver vec SLICES
    python -m paper_2006_14080_amd.profile_driver shard PRECISION [repeats]
    python -m paper_2006_14080_amd.profile_driver nufft [repeats]

The first form calls nudft_forward and the adjoint (nudft_adjoint_prepared,
tables prepared once, as inside a solve) at the 256x256 / 8-coil /
64x512-sample shape `repeats` times, then copies a 256 MiB buffer twice (a
kernel of known traffic: reads 256 MiB, writes 256 MiB) so FETCH_SIZE /
WRITE_SIZE can be calibrated in the same run.

The second runs admm_solve (2 ADMM x 5 CG, FP32) over SLICES slices of
384x384 with one coil and 64 samples, so the NUDFT is negligible and the
solver's memory-bound kernels work on multi-GB arrays (far beyond the 256 MB
Infinity Cache), then copies 1 GiB three times (the plain-copy reference);
it prints the pixel count and the adjoint's partial-image count (from the
library's mri_adjoint_split) that `profsum vecbw` reads.

The third times (HIP events on the calling stream) nudft_forward and
nudft_adjoint on one GPU's share of a k-space decomposition over 8 GPUs
(Sec. IV-A: every coil's samples [0, nk/8)) next to the whole problem, at
the 256x256 / 8-coil benchmark shape and at the 1024x512 / 12-coil /
101x1024-sample shape of Sec. VI, and prints one line per case.
"""
import sys

import numpy as np
import torch

from . import mri, synth


def vector_sweep(slices: int):
    n, nc, spokes, nr = 384, 1, 1, 64
    wl = synth.Workload(f"vec_{slices}x{n}", n, n, nc, spokes, nr, 1e-3, 1.0, 2, 5, batch=slices, seed=900)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    truth = g(np.stack([synth.ellipse_phantom(n, n, 900 + s) for s in range(min(slices, 4))] *
                       ((slices + 3) // 4))[:slices].astype(np.complex64))
    sm = g(synth.coil_maps(n, n, nc))
    tr = g(synth.radial_trajectory(spokes, nr))
    data = mri.nudft_forward(truth, sm, tr)
    shape = mri.shape_of((slices, n, n), sm, tr)
    params = mri.AdmmParams(wl.lam, wl.beta, wl.admm_iters, wl.cg_iters)
    solver = mri.AdmmSolver(shape, params, device=torch.device("cuda"))
    out = torch.empty((slices, n, n), dtype=torch.complex64, device="cuda")
    for _ in range(2):
        solver.solve(sm, tr, data, out=out)
    torch.cuda.synchronize()
    del solver, out, data, truth
    # A device copy of known size (1 GiB read + 1 GiB written) in the same run:
    # the practical bandwidth of a plain read/write stream on this part.
    src = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    planes = mri.adjoint_split(shape)["planes"]
    print(f"profile driver done: npix={slices * n * n} coils={nc} planes={planes}", flush=True)


def _time_ms(fn, repeats: int) -> float:
    # Calls enqueued back to back between two events (the host stays ahead of
    # the GPU), so the figure is device time per call, not host launch gaps.
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(repeats):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / repeats


def shard_timings(prec: int, repeats: int, parts: int = 8):
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    name = mri.PRECISION_NAMES[prec]
    for wl in (synth.ADMM256, synth.TABLE1_1024x512):
        img = g(synth.ellipse_phantom(wl.nx, wl.ny, wl.seed)[None])
        sm = g(synth.coil_maps(wl.nx, wl.ny, wl.nc))
        tr_full = synth.radial_trajectory(wl.n_spokes, wl.n_readout)
        dat_full = synth.random_complex((1, wl.nc, wl.nk), 1)
        lo, hi = synth.kspace_shards(wl.nk, parts)[0]
        for label, tr, dat in (("whole", tr_full, dat_full),
                               (f"shard 1/{parts}", tr_full[lo:hi], dat_full[:, :, lo:hi])):
            gt, gd = g(tr), g(dat)
            nk = tr.shape[0]
            y = torch.empty((1, wl.nc, nk), dtype=torch.complex64, device="cuda")
            x = torch.empty((1, wl.ny, wl.nx), dtype=torch.complex64, device="cuda")
            plan = mri.AdjointPlan(sm, gt, wl.ny, wl.nx, precision=prec)
            fwd = lambda: mri.nudft_forward(img, sm, gt, precision=prec, out=y)
            adj = lambda: plan(gd, out=x)
            fwd(), adj()
            tf, ta = _time_ms(fwd, repeats), _time_ms(adj, repeats)
            flop = 8.0 * nk * wl.nx * wl.ny * wl.nc
            print(f"{name:7s} {wl.nx}x{wl.ny} c{wl.nc} nk={nk:6d} {label:9s} "
                  f"fwd {tf:8.3f} ms {flop / tf / 1e9:6.1f} TFLOP/s   "
                  f"adj {ta:8.3f} ms {flop / ta / 1e9:6.1f} TFLOP/s", flush=True)
    print("profile driver done", flush=True)


def nufft_timings(repeats: int):
    """NUFFT operator (width 6, oversampling 2) beside the dense NUDFT (FP32,
    BF16x3) at the 256x256 / 8-coil / 64x512-sample and the 1024x512 /
    12-coil / 101x1024-sample shapes: HIP-event times per call (plan and
    phase tables built once, as inside a solve) and the NUFFT's plan time."""
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for wl in (synth.ADMM256, synth.TABLE1_1024x512):
        img = g(synth.ellipse_phantom(wl.nx, wl.ny, wl.seed)[None])
        sm = g(synth.coil_maps(wl.nx, wl.ny, wl.nc))
        tr = g(synth.radial_trajectory(wl.n_spokes, wl.n_readout))
        dat = g(synth.random_complex((1, wl.nc, wl.nk), 1))
        y = torch.empty((1, wl.nc, wl.nk), dtype=torch.complex64, device="cuda")
        x = torch.empty((1, wl.ny, wl.nx), dtype=torch.complex64, device="cuda")
        shape = f"{wl.nx}x{wl.ny} c{wl.nc} nk={wl.nk}"
        tp = _time_ms(lambda: mri.NufftPlan(sm, tr, wl.ny, wl.nx), 2)
        plan = mri.NufftPlan(sm, tr, wl.ny, wl.nx)
        tf = _time_ms(lambda: plan.forward(img, out=y), repeats)
        ta = _time_ms(lambda: plan.adjoint(dat, out=x), repeats)
        print(f"nufft   {shape}  fwd {tf:8.3f} ms  adj {ta:8.3f} ms  plan {tp:8.3f} ms", flush=True)
        for prec in (mri.FP32, mri.BF16X3):
            adj = mri.AdjointPlan(sm, tr, wl.ny, wl.nx, precision=prec)
            tf = _time_ms(lambda: mri.nudft_forward(img, sm, tr, precision=prec, out=y), max(2, repeats // 4))
            ta = _time_ms(lambda: adj(dat, out=x), max(2, repeats // 4))
            print(f"{mri.PRECISION_NAMES[prec]:7s} {shape}  fwd {tf:8.3f} ms  adj {ta:8.3f} ms", flush=True)
    print("profile driver done", flush=True)


def main(argv):
    if len(argv) > 1 and argv[1] == "vec":
        vector_sweep(int(argv[2]))
        return
    if len(argv) > 1 and argv[1] == "nufft":
        nufft_timings(int(argv[2]) if len(argv) > 2 else 20)
        return
    if len(argv) > 1 and argv[1] == "shard":
        shard_timings(mri.PRECISIONS[argv[2]], int(argv[3]) if len(argv) > 3 else 5)
        return
    prec = mri.PRECISIONS[argv[1]] if len(argv) > 1 else mri.FP32
    n = int(argv[2]) if len(argv) > 2 else 2
    wl = synth.ADMM256
    p = synth.make_problem(wl)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    img, sm, tr = g(p.truth), g(p.smaps), g(p.traj)
    dat = g(synth.random_complex((1, wl.nc, wl.nk), 1))
    plan = mri.AdjointPlan(sm, tr, wl.ny, wl.nx, precision=prec)   # phase tables once, as in a solve
    for _ in range(n):
        mri.nudft_forward(img, sm, tr, precision=prec)
        plan(dat)
    torch.cuda.synchronize()
    src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("profile driver done", flush=True)


if __name__ == "__main__":
    main(sys.argv)
