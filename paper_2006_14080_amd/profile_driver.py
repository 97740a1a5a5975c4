"""Fixed workload for hardware-counter runs (rocprofv3 --pmc).

    python -m paper_2006_14080_amd.profile_driver [fp32|bf16x3] [repeats]

Calls nudft_forward and nudft_adjoint at the 256x256 / 8-coil / 64x512-sample
shape `repeats` times, then copies a 256 MiB buffer twice (a kernel of known
traffic: reads 256 MiB, writes 256 MiB) so FETCH_SIZE / WRITE_SIZE can be
calibrated in the same run.
"""
import sys

import numpy as np
import torch

from . import mri, synth


def main(argv):
    prec = mri.PRECISIONS[argv[1]] if len(argv) > 1 else mri.FP32
    n = int(argv[2]) if len(argv) > 2 else 2
    wl = synth.ADMM256
    p = synth.make_problem(wl)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    img, sm, tr = g(p.truth), g(p.smaps), g(p.traj)
    dat = g(synth.random_complex((1, wl.nc, wl.nk), 1))
    for _ in range(n):
        mri.nudft_forward(img, sm, tr, precision=prec)
        mri.nudft_adjoint(dat, sm, tr, wl.ny, wl.nx, precision=prec)
    torch.cuda.synchronize()
    src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    print("profile driver done", flush=True)


if __name__ == "__main__":
    main(sys.argv)
