"""Measure how far the FP64 oracle's own ADMM image moves when its operator
outputs carry FP32-sized errors, and store the numbers the GPU image bars are
derived from.

    python tests/golden/make_tolerances.py

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
form's workload).  Writes tolerances.json next to this script.
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


def perturbed_admm(data, smaps, traj, wl, perturb):
    """The oracle's ADMM with `perturb` applied to every F and F^H output."""
    def fwd(v):
        return perturb(nudft.forward(v, smaps, traj))

    def adj(u):
        return perturb(nudft.adjoint(u, smaps, traj))

    def apply_a(v):
        return adj(fwd(v)) + 0.5 * wl.beta * tv.tv_adjoint(tv.tv_forward(v))

    return admm.admm(data, smaps, traj, wl.lam, wl.beta, wl.admm_iters, wl.cg_iters, rtol=wl.rtol,
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


# Per-operator relative errors of the GPU forms (forward and adjoint against
# the oracle on an 80x72, 5-coil, 2500-sample problem): FP32 2.7e-7 / 6.3e-7,
# FP16x3 2.1e-7 / 4.0e-7, BF16x3 3.8e-6 / 3.8e-6.
FP32_EPS = (1e-7, 1e-6)
BF16X3_EPS = (4e-6,)
SEEDS = (1, 2, 3)


def main():
    t0 = time.time()
    res = {
        "admm32": case(synth.ADMM32, FP32_EPS + BF16X3_EPS, SEEDS + (4, 5)),
        "table1_128x64": case(synth.TABLE1_128x64, FP32_EPS, SEEDS),
    }
    res["seconds"] = time.time() - t0
    out = os.path.join(HERE, "tolerances.json")
    with open(out, "w") as f:
        json.dump(res, f, indent=1)
    print(f"wrote {out} ({res['seconds']:.0f} s)")


if __name__ == "__main__":
    main()
