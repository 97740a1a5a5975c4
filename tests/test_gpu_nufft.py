"""The NUFFT operator (nufft_prepare / nufft_forward / nufft_adjoint) on the
GPU through the C ABI.

* against the FP64 oracle of the same algorithm (oracle/nufft.py: same grid,
  kernel, deapodisation): the FP32 arithmetic bar of the dense operators,
  1e-5 relative, over whole outputs, including the 256x256 / 8-coil /
  64x512-sample benchmark shape;
* against the exact NUDFT (oracle/nudft.py): within the NUFFT's stated
  approximation bound (width 6: 1e-5, width 7: 1e-6, pinned on the CPU in
  test_oracle_nufft.py) plus FP32 rounding;
* the adjoint identity, bitwise run-to-run reproducibility (the spreading
  gathers samples in a fixed order), batches with per-slice trajectories and
  maps, odd and non-square grids, and a single sample.
"""
import numpy as np
import pytest
import torch

from oracle import nudft as onudft
from oracle import nufft as onufft
from paper_2006_14080_amd import mri, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(nx, ny, nc, nk=None, spokes=None, nr=None, seed=3):
    img = synth.ellipse_phantom(nx, ny, seed).astype(np.complex64)
    sm = (synth.coil_maps(nx, ny, nc) + 0.2 * synth.random_complex((nc, ny, nx), seed + 1)).astype(np.complex64)
    traj = synth.radial_trajectory(spokes, nr) if spokes else synth.random_trajectory(nk, seed + 2)
    dat = synth.random_complex((nc, traj.shape[0]), seed + 3)
    return img, sm, traj, dat


@pytest.mark.parametrize("nx,ny,nc,width,sigma", [(32, 32, 2, 6, 2.0), (45, 37, 3, 6, 2.0), (64, 20, 4, 7, 2.0),
                                                  (17, 29, 1, 4, 1.5), (40, 40, 9, 8, 2.5)])
def test_matches_oracle_nufft(nx, ny, nc, width, sigma):
    img, sm, traj, dat = _case(nx, ny, nc, nk=700)
    plan = mri.NufftPlan(_gpu(sm), _gpu(traj), ny, nx, width=width, sigma=sigma)
    op = onufft.Plan(nx, ny, traj, width=width, sigma=sigma)
    y = plan.forward(_gpu(img[None])).cpu().numpy()[0]
    assert _rel(y, onufft.forward(img, sm, op)) <= 1e-5
    x = plan.adjoint(_gpu(dat[None])).cpu().numpy()[0]
    assert _rel(x, onufft.adjoint(dat, sm, op)) <= 1e-5


@pytest.mark.parametrize("width,bound", [(6, 1e-5), (7, 2e-6)])
def test_approximates_the_exact_nudft(width, bound):
    nx, ny, nc = 48, 40, 3
    img, sm, traj, dat = _case(nx, ny, nc, spokes=24, nr=96)
    plan = mri.NufftPlan(_gpu(sm), _gpu(traj), ny, nx, width=width)
    y = plan.forward(_gpu(img[None])).cpu().numpy()[0]
    assert _rel(y, onudft.forward(img, sm, traj)) <= bound
    x = plan.adjoint(_gpu(dat[None])).cpu().numpy()[0]
    assert _rel(x, onudft.adjoint(dat, sm, traj)) <= bound


def test_benchmark_shape_against_oracle_nufft_and_sampled_nudft():
    wl = synth.ADMM256
    p = synth.make_problem(wl)
    plan = mri.NufftPlan(_gpu(p.smaps), _gpu(p.traj), wl.ny, wl.nx)
    op = onufft.Plan(wl.nx, wl.ny, p.traj)
    y = plan.forward(_gpu(p.truth)).cpu().numpy()[0]
    assert _rel(y, onufft.forward(p.truth[0], p.smaps, op)) <= 1e-5
    # exact NUDFT on sampled outputs (the oracle's full forward takes seconds here)
    rng = np.random.default_rng(0)
    gi, ki = rng.integers(0, wl.nc, 200), rng.integers(0, wl.nk, 200)
    ref = onudft.forward_samples(p.truth[0], p.smaps, p.traj, gi, ki)
    assert _rel(y[gi, ki], ref) <= 1e-5
    dat = synth.random_complex((wl.nc, wl.nk), 5)
    x = plan.adjoint(_gpu(dat[None])).cpu().numpy()[0]
    assert _rel(x, onufft.adjoint(dat, p.smaps, op)) <= 1e-5
    yi, xi = rng.integers(0, wl.ny, 100), rng.integers(0, wl.nx, 100)
    assert _rel(x[yi, xi], onudft.adjoint_pixels(dat, p.smaps, p.traj, yi, xi)) <= 1e-5


def test_adjoint_identity_and_reproducibility():
    nx, ny, nc = 64, 48, 4
    img, sm, traj, dat = _case(nx, ny, nc, nk=3000)
    plan = mri.NufftPlan(_gpu(sm), _gpu(traj), ny, nx)
    xr = synth.random_complex((1, ny, nx), 11)
    y = plan.forward(_gpu(xr)).cpu().numpy()
    x = plan.adjoint(_gpu(dat[None])).cpu().numpy()
    lhs, rhs = np.vdot(y.astype(np.complex128), dat[None]), np.vdot(xr.astype(np.complex128), x)
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    for _ in range(3):
        assert np.array_equal(plan.forward(_gpu(xr)).cpu().numpy(), y)
        assert np.array_equal(plan.adjoint(_gpu(dat[None])).cpu().numpy(), x)


def test_batch_with_per_slice_trajectories_and_maps():
    nx, ny, nc, nk, nb = 30, 26, 3, 500, 3
    imgs = np.stack([synth.ellipse_phantom(nx, ny, 20 + b) for b in range(nb)]).astype(np.complex64)
    maps = np.stack([synth.random_complex((nc, ny, nx), 30 + b) for b in range(nb)])
    trajs = np.stack([synth.random_trajectory(nk, 40 + b) for b in range(nb)])
    dats = np.stack([synth.random_complex((nc, nk), 50 + b) for b in range(nb)])
    plan = mri.NufftPlan(_gpu(maps), _gpu(trajs), ny, nx, batch=nb)
    y = plan.forward(_gpu(imgs)).cpu().numpy()
    x = plan.adjoint(_gpu(dats)).cpu().numpy()
    for b in range(nb):
        op = onufft.Plan(nx, ny, trajs[b])
        assert _rel(y[b], onufft.forward(imgs[b], maps[b], op)) <= 1e-5
        assert _rel(x[b], onufft.adjoint(dats[b], maps[b], op)) <= 1e-5
        one = mri.NufftPlan(_gpu(maps[b]), _gpu(trajs[b]), ny, nx)
        assert np.array_equal(one.forward(_gpu(imgs[b:b + 1])).cpu().numpy()[0], y[b])
        assert np.array_equal(one.adjoint(_gpu(dats[b:b + 1])).cpu().numpy()[0], x[b])


def test_single_sample_and_zero_input():
    nx, ny, nc = 16, 16, 2
    sm = synth.coil_maps(nx, ny, nc)
    traj = np.array([[0.3, -1.1]])
    plan = mri.NufftPlan(_gpu(sm), _gpu(traj), ny, nx)
    img = synth.random_complex((1, ny, nx), 1)
    y = plan.forward(_gpu(img)).cpu().numpy()[0]
    assert _rel(y, onudft.forward(img[0], sm, traj)) <= 1e-5
    assert np.all(plan.adjoint(torch.zeros((1, nc, 1), dtype=torch.complex64, device=DEV)).cpu().numpy() == 0)
