"""nudft_forward_noalloc (the forward for callers that cannot allocate)
through the C ABI: same output as nudft_forward, bit for bit, on two calls in
a row (the second with a smaller input, so the shared scratch still holds the
first call's larger contents), in every precision form; shapes beyond the
scratch are refused on the host."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2006_14080_amd import mri, synth

pytestmark = pytest.mark.gpu


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _inputs(nx, ny, nc, spokes, nr, nb, seed):
    truth = np.stack([synth.ellipse_phantom(nx, ny, seed + b) for b in range(nb)])
    return _gpu(truth), _gpu(synth.coil_maps(nx, ny, nc)), _gpu(synth.radial_trajectory(spokes, nr))


def _noalloc(img, sm, tr, prec):
    lib = mri.load()      # sets the entry point's argument types
    sh = mri.shape_of(img.shape, sm, tr)
    out = torch.full((sh.batch, sh.ncoils, sh.nk), float("nan"), dtype=torch.complex64, device="cuda")
    rc = lib.nudft_forward_noalloc(ctypes.byref(sh), ctypes.c_void_p(img.data_ptr()),
                                   ctypes.c_void_p(sm.data_ptr()), ctypes.c_void_p(tr.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), prec,
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, mri.ERRORS.get(rc, rc)
    return out


@pytest.mark.parametrize("prec", [mri.FP32, mri.BF16X3, mri.FP16X3])
def test_noalloc_forward_matches_forward(prec):
    # a large call, then a smaller one (odd, non-square, ragged sample tail)
    for nx, ny, nc, spokes, nr, nb in [(256, 256, 8, 64, 512, 2), (45, 37, 3, 7, 90, 1)]:
        img, sm, tr = _inputs(nx, ny, nc, spokes, nr, nb, 11)
        want = mri.nudft_forward(img, sm, tr, precision=prec)
        got = _noalloc(img, sm, tr, prec)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (nx, ny, nc)


def test_noalloc_refuses_shapes_beyond_its_scratch():
    lib = mri.load()
    cap = lib.mri_noalloc_scratch_bytes()
    assert cap == 64 << 20
    sh = mri.make_shape(1024, 1024, 16, 1024)        # 128 MiB of coil-weighted images
    assert mri.workspace_bytes(sh, mri.OP_FORWARD) > cap
    fake = ctypes.c_void_p(0x1000)                   # never dereferenced: refused first
    rc = lib.nudft_forward_noalloc(ctypes.byref(sh), fake, fake, fake, fake, 0, None)
    assert rc == -2
