"""One GPU's share of the k-space decomposition (Sec. IV-A), through the C ABI.

In the paper's decomposition core p of P holds the samples
[p*nk/P, (p+1)*nk/P) of every coil and that range of the trajectory, while
the image and the coil maps are replicated.  Two facts make the scheme exact,
and these tests check both on the per-core kernels:

* the forward of a sample range is that range of the whole forward (each
  output sample depends only on its own trajectory point), so the kernels
  must give it bit for bit;
* the adjoint is a sum over samples, so the whole adjoint, and the whole
  normal operator F^H F of each CG step, is the sum over cores of their
  partial results (the one image-sized all-reduce per application of A,
  Alg. 3).  The per-core sums are added here in FP64 on the host, standing in
  for that exchange; they must match the whole-problem result and the FP64
  oracle to the 1e-5 per-operator bar.

Shapes: the 256x256 / 8-coil / 64x512-sample benchmark problem split over 8
cores (4096 samples per coil each, whole tiles) and over 7 (ragged ranges),
and the 1024x512 / 12-coil / 101x1024-sample problem of Sec. VI, whose
one-of-eight share is checked on sampled outputs.
"""
import numpy as np
import pytest
import torch

from oracle import nudft as onudft
from paper_2006_14080_amd import mri, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = 1e-5
PRECS = [mri.FP32, mri.BF16X3, mri.FP16X3]


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _bench_problem():
    wl = synth.ADMM256
    img = synth.ellipse_phantom(wl.nx, wl.ny, wl.seed)[None] + synth.random_complex((1, wl.ny, wl.nx), 501) * np.complex64(0.05)
    sm = synth.coil_maps(wl.nx, wl.ny, wl.nc)
    tr = synth.radial_trajectory(wl.n_spokes, wl.n_readout)
    dat = synth.random_complex((1, wl.nc, wl.nk), 502)
    return wl, img.astype(np.complex64), sm, tr, dat


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("parts", [8, 7])
def test_forward_of_a_sample_range_is_that_range_of_the_whole(parts, prec):
    wl, img, sm, tr, _ = _bench_problem()
    gi, gs = _gpu(img), _gpu(sm)
    whole = mri.nudft_forward(gi, gs, _gpu(tr), precision=prec)
    for lo, hi in synth.kspace_shards(wl.nk, parts):
        part = mri.nudft_forward(gi, gs, _gpu(tr[lo:hi]), precision=prec)
        assert torch.equal(part, whole[:, :, lo:hi]), (lo, hi)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("parts", [8, 7])
def test_adjoints_of_the_sample_ranges_sum_to_the_whole(parts, prec):
    wl, _, sm, tr, dat = _bench_problem()
    gs = _gpu(sm)
    whole = mri.nudft_adjoint(_gpu(dat), gs, _gpu(tr), wl.ny, wl.nx, precision=prec).cpu().numpy()[0]
    total = np.zeros((wl.ny, wl.nx), np.complex128)
    rng = np.random.default_rng(503)
    for p, (lo, hi) in enumerate(synth.kspace_shards(wl.nk, parts)):
        part = mri.nudft_adjoint(_gpu(dat[:, :, lo:hi]), gs, _gpu(tr[lo:hi]), wl.ny, wl.nx,
                                 precision=prec).cpu().numpy()[0]
        total += part
        if p in (0, parts - 1):
            # parity of the per-core operator itself at its real shape
            rows, cols = rng.integers(0, wl.ny, 32), rng.integers(0, wl.nx, 32)
            ref = onudft.adjoint_pixels(dat[0][:, lo:hi], sm, tr[lo:hi], rows, cols)
            assert _rel(part[rows, cols], ref) <= TOL
    assert _rel(total, whole) <= TOL
    rows, cols = rng.integers(0, wl.ny, 48), rng.integers(0, wl.nx, 48)
    assert _rel(total[rows, cols], onudft.adjoint_pixels(dat[0], sm, tr, rows, cols)) <= TOL


@pytest.mark.parametrize("prec", PRECS)
def test_normal_operator_is_the_sum_over_cores(prec):
    # F^H F x, the operator applied on every CG step: each core applies its
    # own F_p^H F_p and the results are summed (the per-step exchange).
    wl, img, sm, tr, _ = _bench_problem()
    gi, gs = _gpu(img), _gpu(sm)

    def normal(t):
        y = mri.nudft_forward(gi, gs, t, precision=prec)
        return mri.nudft_adjoint(y, gs, t, wl.ny, wl.nx, precision=prec).cpu().numpy()[0]

    whole = normal(_gpu(tr))
    total = np.zeros((wl.ny, wl.nx), np.complex128)
    for lo, hi in synth.kspace_shards(wl.nk, 8):
        total += normal(_gpu(tr[lo:hi]))
    assert _rel(total, whole) <= TOL


@pytest.mark.parametrize("prec", PRECS)
def test_large_image_one_core_share_sampled(prec):
    # 1024x512, 12 coils: the whole problem and one core's share of 8
    # (12928 samples per coil), on outputs the oracle computes one by one.
    wl = synth.TABLE1_1024x512
    rng = np.random.default_rng(504)
    img = synth.random_complex((1, wl.ny, wl.nx), 505)
    sm = synth.coil_maps(wl.nx, wl.ny, wl.nc)
    tr = synth.radial_trajectory(wl.n_spokes, wl.n_readout)
    dat = synth.random_complex((1, wl.nc, wl.nk), 506)
    gi, gs = _gpu(img), _gpu(sm)
    lo, hi = synth.kspace_shards(wl.nk, 8)[3]
    for a, b in ((0, wl.nk), (lo, hi)):
        t = _gpu(tr[a:b])
        f = mri.nudft_forward(gi, gs, t, precision=prec).cpu().numpy()[0]
        x = mri.nudft_adjoint(_gpu(dat[:, :, a:b]), gs, t, wl.ny, wl.nx, precision=prec).cpu().numpy()[0]
        coils, ks = rng.integers(0, wl.nc, 48), rng.integers(0, b - a, 48)
        ks[:2] = [0, b - a - 1]
        assert _rel(f[coils, ks], onudft.forward_samples(img[0], sm, tr[a:b], coils, ks)) <= TOL
        rows, cols = rng.integers(0, wl.ny, 32), rng.integers(0, wl.nx, 32)
        rows[:2], cols[:2] = [0, wl.ny - 1], [wl.nx - 1, 0]
        assert _rel(x[rows, cols], onudft.adjoint_pixels(dat[0][:, a:b], sm, tr[a:b], rows, cols)) <= TOL
