"""Write the FP64 oracle's reconstruction of two slices of the 32-slice
384x384 batch workload at reduced counts.

    python tests/golden/make_slices384_golden.py

Calls only the oracle and the seeded input generators.  Slices 0 and 31 of the
batch (384x384, 16 coils, 128 golden-angle spokes x 768 samples, lambda 5e-4,
beta 1): data = oracle F(phantom) + noise (rounded to complex64, as the GPU
receives it), then the oracle's ADMM with 2 ADMM x 2 CG steps (13 NUDFT
applications per slice).  Writes slices384_oracle.npz: the k-space data each
slice was solved for (complex64 [2][coils][nk], 25 MB), the complex64 images
and the solve counters.  About 8 minutes on 8 cores.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import admm, nudft  # noqa: E402
from paper_2006_14080_amd import synth  # noqa: E402

SLICES = (0, 31)
ADMM_ITERS, CG_ITERS = 2, 2


def slice_data(wl, b, smaps, traj):
    """k-space data of slice b: oracle F(phantom) + noise, rounded to complex64."""
    return (nudft.forward(synth.slice_phantom(wl, b), smaps, traj) + synth.slice_noise(wl, b)).astype(np.complex64)


def main():
    wl = synth.SLICES384
    smaps = synth.coil_maps(wl.nx, wl.ny, wl.nc)
    traj = synth.radial_trajectory(wl.n_spokes, wl.n_readout)
    images, counts, datas = [], [], []
    t0 = time.time()
    for b in SLICES:
        data = slice_data(wl, b, smaps, traj)
        res = admm.admm(data, smaps, traj, wl.lam, wl.beta, ADMM_ITERS, CG_ITERS)
        images.append(res.image.astype(np.complex64))
        counts.append((res.admm_iters, res.cg_steps))
        datas.append(data)
        print(f"slice {b}: {res.admm_iters} ADMM, {res.cg_steps} CG, {time.time() - t0:.0f} s", flush=True)
    out = os.path.join(HERE, "slices384_oracle.npz")
    np.savez_compressed(out, slices=np.array(SLICES), data=np.stack(datas), images=np.stack(images),
                        counts=np.array(counts), admm_iters=ADMM_ITERS, cg_iters=CG_ITERS,
                        seconds=time.time() - t0)
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
