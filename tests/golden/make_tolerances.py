"""Measure how far the FP64 oracle's own ADMM image moves when its operator
outputs carry FP32-sized errors, and store the numbers the GPU image bars are
derived from.

    python tests/golden/make_tolerances.py [case ...]      (default: admm32 table1_128x64)

Calls only the oracle and the seeded input generators.  For each case the
oracle runs once exactly and then with every output of F and F^H perturbed
(the F^H d of the right-hand side, and both operators inside A = F^H F +
(beta/2) Theta^H Theta):
  * "c64": each output rounded to complex64, as a GPU operator's output is
    stored;
  * "noise": each output v replaced by v + eps ||v|| g / ||g|| with g a fresh
    complex Gaussian vector, i.e. a relative L2 operator error eps, at the
    per-operator errors measured for the GPU forms (about 3e-7 in FP32 and
    FP16x3, 4e-6 in BF16x3), over several seeds.
The image shift is the NRMSE of the perturbed image against the exact one.
Cases: the 128x64 / 12-coil / 13x128 Table I problem (Sec. V; lambda 1e-7
leaves its 20-step CG an almost unregularised least-squares solve) and the
32x32 / 4-coil / 16x64 problem at 10 ADMM x 3 CG (the BF16x3 precision
form's workload), each solved exactly first; and, at the BF16x3 operator
error only, the three problems whose oracle reconstructions are stored beside
this script (written by make_admm256_golden.py, make_slices384_golden.py and
make_table1_large_golden.py from the oracle alone), which serve as the exact
images: the 256x256 benchmark at 30 ADMM x 5 CG (about 12 minutes per solve
on 8 cores), slice 0 of the 32 x 384x384 batch at 2 x 2 and the 1024x512
Table I problem at 1 x 2.  Results are merged into tolerances.json next to
this script, one key per case.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import admm, nudft, tv  # noqa: E402
from paper_2006_14080_amd import synth  # noqa: E402


def perturbed_admm(data, smaps, traj, wl, perturb, counts=None):
    """The oracle's ADMM with `perturb` applied to every F and F^H output
    (at the workload's iteration counts, or at counts = (admm, cg))."""
    def fwd(v):
        return perturb(nudft.forward(v, smaps, traj))

    def adj(u):
        return perturb(nudft.adjoint(u, smaps, traj))

    def apply_a(v):
        return adj(fwd(v)) + 0.5 * wl.beta * tv.tv_adjoint(tv.tv_forward(v))

    na, ncg = counts if counts else (wl.admm_iters, wl.cg_iters)
    return admm.admm(data, smaps, traj, wl.lam, wl.beta, na, ncg, rtol=wl.rtol,
                     atol=wl.atol, apply_a=apply_a, adjoint=adj)


def round_c64(v):
    return np.asarray(v).astype(np.complex64).astype(np.complex128)


def rel_noise(eps, seed):
    rng = np.random.default_rng(seed)

    def f(v):
        g = rng.standard_normal(v.shape) + 1j * rng.standard_normal(v.shape)
        return v + eps * np.linalg.norm(v) * g / np.linalg.norm(g)
    return f


def nrmse(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def case(wl, eps_list, seeds):
    p = synth.make_problem(wl)
    data = (nudft.forward(p.truth[0], p.smaps, p.traj) + p.noise[0]).astype(np.complex64)
    exact = perturbed_admm(data, p.smaps, p.traj, wl, lambda v: v)
    out = {"workload": wl.name, "admm_iters": exact.admm_iters, "cg_steps": exact.cg_steps}
    c64 = perturbed_admm(data, p.smaps, p.traj, wl, round_c64)
    out["c64"] = nrmse(c64.image, exact.image)
    out["noise"] = {}
    for eps in eps_list:
        shifts = [nrmse(perturbed_admm(data, p.smaps, p.traj, wl, rel_noise(eps, s)).image, exact.image)
                  for s in seeds]
        out["noise"][f"{eps:.0e}"] = shifts
        print(f"{wl.name} eps {eps:.0e}: {['%.3e' % v for v in shifts]}", flush=True)
    out["max_shift"] = max([out["c64"]] + [v for s in out["noise"].values() for v in s])
    print(f"{wl.name}: c64 {out['c64']:.3e}, max {out['max_shift']:.3e}", flush=True)
    return out


def stored_case(name, wl, smaps, traj, data, exact, counts, eps_list, seeds):
    """Shifts against an oracle reconstruction stored by a golden script."""
    data = np.asarray(data).astype(np.complex64)
    exact = np.asarray(exact).astype(np.complex128)
    out = {"workload": wl.name, "counts": list(counts), "reference": name, "noise": {}}
    t0 = time.time()
    for eps in eps_list:
        shifts = []
        for s in seeds:
            shifts.append(nrmse(perturbed_admm(data, smaps, traj, wl, rel_noise(eps, s), counts).image, exact))
            print(f"{wl.name} eps {eps:.0e} seed {s}: {shifts[-1]:.3e} ({time.time() - t0:.0f} s)", flush=True)
        out["noise"][f"{eps:.0e}"] = shifts
    out["max_shift"] = max(v for s in out["noise"].values() for v in s)
    return out


def admm256_bf16x3():
    g = np.load(os.path.join(HERE, "admm256_oracle.npz"))
    wl = synth.ADMM256
    p = synth.make_problem(wl)
    return stored_case("admm256_oracle.npz", wl, p.smaps, p.traj, g["data"], g["image"],
                       (wl.admm_iters, wl.cg_iters), BF16X3_EPS, SEEDS)


def slices384_bf16x3():
    g = np.load(os.path.join(HERE, "slices384_oracle.npz"))
    wl = synth.SLICES384
    i = 0                                       # slice g["slices"][0]
    return stored_case(f"slices384_oracle.npz slice {int(g['slices'][i])}", wl,
                       synth.coil_maps(wl.nx, wl.ny, wl.nc), synth.radial_trajectory(wl.n_spokes, wl.n_readout),
                       g["data"][i], g["images"][i], (int(g["admm_iters"]), int(g["cg_iters"])), BF16X3_EPS, SEEDS)


def table1_large_bf16x3():
    g = np.load(os.path.join(HERE, "table1_large_oracle.npz"))
    wl = synth.TABLE1_1024x512
    return stored_case("table1_large_oracle.npz", wl, synth.coil_maps(wl.nx, wl.ny, wl.nc),
                       synth.radial_trajectory(wl.n_spokes, wl.n_readout), g["data"], g["image"],
                       (int(g["admm_max"]), int(g["cg_max"])), BF16X3_EPS, SEEDS)


# Per-operator relative errors of the GPU forms (forward and adjoint against
# the oracle on an 80x72, 5-coil, 2500-sample problem): FP32 2.7e-7 / 6.3e-7,
# FP16x3 2.1e-7 / 4.0e-7, BF16x3 3.8e-6 / 3.8e-6.
FP32_EPS = (1e-7, 1e-6)
BF16X3_EPS = (4e-6,)
SEEDS = (1, 2, 3)


CASES = {
    "admm32": lambda: case(synth.ADMM32, FP32_EPS + BF16X3_EPS, SEEDS + (4, 5)),
    "table1_128x64": lambda: case(synth.TABLE1_128x64, FP32_EPS, SEEDS),
    "admm256_bf16x3": admm256_bf16x3,
    "slices384_bf16x3": slices384_bf16x3,
    "table1_large_bf16x3": table1_large_bf16x3,
}


def main(names):
    out = os.path.join(HERE, "tolerances.json")
    for name in names or ["admm32", "table1_128x64"]:
        t0 = time.time()
        r = CASES[name]()
        r["seconds"] = time.time() - t0
        res = json.load(open(out)) if os.path.exists(out) else {}
        res.pop("seconds", None)
        res[name] = r
        with open(out, "w") as f:
            json.dump(res, f, indent=1)
        print(f"{name}: max shift {r['max_shift']:.3e}; wrote {out} ({r['seconds']:.0f} s)", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
