"""Write the FP64 oracle's reconstruction of the large-image case of Sec. VI
at reduced counts.

    python tests/golden/make_table1_large_golden.py

Calls only the oracle and the seeded input generators.  The 1024x512 grid,
12 coils, 101 spokes x 1024 samples, with the Table I settings (lambda 1e-7,
beta 1, rtol 1e-4, atol 1e-6) but 1 ADMM x 2 CG steps (7 NUDFT applications,
5.2e12 flop each): data = oracle F(phantom) + noise (rounded to complex64),
then the oracle's ADMM.  Writes table1_large_oracle.npz: the k-space data it
solved for (complex64 [coils][nk], 10 MB), the complex64 image, the counters
and the data residual ||F(image) - d|| / ||d||.  About 6 minutes on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import admm, nudft  # noqa: E402
from paper_2006_14080_amd import synth  # noqa: E402

ADMM_ITERS, CG_ITERS = 1, 2


def make_data(wl, smaps, traj):
    """k-space data: oracle F(phantom) + noise, rounded to complex64."""
    return (nudft.forward(synth.slice_phantom(wl, 0), smaps, traj) + synth.slice_noise(wl, 0)).astype(np.complex64)


def main():
    wl = synth.TABLE1_1024x512
    smaps = synth.coil_maps(wl.nx, wl.ny, wl.nc)
    traj = synth.radial_trajectory(wl.n_spokes, wl.n_readout)
    t0 = time.time()
    data = make_data(wl, smaps, traj)
    print(f"data formed, {time.time() - t0:.0f} s", flush=True)
    res = admm.admm(data, smaps, traj, wl.lam, wl.beta, ADMM_ITERS, CG_ITERS, rtol=wl.rtol, atol=wl.atol)
    print(f"{res.admm_iters} ADMM, {res.cg_steps} CG, {time.time() - t0:.0f} s", flush=True)
    d = data.astype(np.complex128)
    resid = np.linalg.norm(nudft.forward(res.image, smaps, traj) - d) / np.linalg.norm(d)
    out = os.path.join(HERE, "table1_large_oracle.npz")
    np.savez_compressed(out, data=data, image=res.image.astype(np.complex64), admm_iters=res.admm_iters,
                        cg_steps=res.cg_steps, alpha=res.alpha, tau=res.tau, resid=resid,
                        admm_max=ADMM_ITERS, cg_max=CG_ITERS, seconds=time.time() - t0)
    print(f"wrote {out}: residual {resid:.4e}")


if __name__ == "__main__":
    main()
