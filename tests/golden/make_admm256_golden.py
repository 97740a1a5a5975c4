"""Write the FP64 oracle's reconstruction of the 256x256 benchmark problem.

    python tests/golden/make_admm256_golden.py

Calls only the oracle and the seeded input generators: data = oracle F(phantom)
+ noise (rounded to complex64, as the GPU receives it), then the oracle's ADMM
with the workload's parameters (30 ADMM x 5 CG, lambda 1e-3, beta 1).  Writes
admm256_oracle.npz: the k-space data it solved for (complex64 [coils][nk]),
the complex64 image and the solve's counters.  Takes about 12 minutes on 8
cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import admm, nudft  # noqa: E402
from paper_2006_14080_amd import synth  # noqa: E402


def main():
    wl = synth.ADMM256
    p = synth.make_problem(wl)
    data = (nudft.forward(p.truth[0], p.smaps, p.traj) + p.noise[0]).astype(np.complex64)
    t0 = time.time()
    res = admm.admm(data, p.smaps, p.traj, wl.lam, wl.beta, wl.admm_iters, wl.cg_iters)
    dt = time.time() - t0
    out = os.path.join(HERE, "admm256_oracle.npz")
    np.savez_compressed(out, data=data, image=res.image.astype(np.complex64), admm_iters=res.admm_iters,
                        cg_steps=res.cg_steps, alpha=res.alpha, tau=res.tau, seconds=dt)
    print(f"wrote {out}: {res.admm_iters} ADMM, {res.cg_steps} CG steps, {dt:.0f} s")


if __name__ == "__main__":
    main()
