"""GPU parity of the single operators (nudft_forward, nudft_adjoint, tv_*)
against the FP64 oracle, through the C ABI.

Bar: relative L2 error <= 1e-5 per NUDFT (element by element over the whole
output), in FP32 and in the split forms (BF16x3, FP16x3); TV transforms are
exact up to one FP32 rounding per element.  The FP16x3 form is also held to
1e-6 and checked over extreme input scales (its operands are rescaled by
powers of two into fp16's range).
Sizes span several tiles (64 samples / 256 rows for the forward, 64 x 32
pixels and 8-coil groups for the adjoint) with ragged tails; full-size
shapes are checked on sampled outputs that the oracle computes one by one.
"""
import numpy as np
import pytest
import torch

from oracle import nudft as onudft
from oracle import tv as otv
from paper_2006_14080_amd import mri, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
TOL = 1e-5


def rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _inputs(nx, ny, nc, nk, batch, seed, traj_batched=False, smaps_batched=False):
    img = synth.random_complex((batch, ny, nx), seed)
    sm = synth.random_complex((batch, nc, ny, nx) if smaps_batched else (nc, ny, nx), seed + 1)
    if traj_batched:
        tr = np.stack([synth.random_trajectory(nk, seed + 2 + b) for b in range(batch)])
    else:
        tr = synth.random_trajectory(nk, seed + 2)
    dat = synth.random_complex((batch, nc, nk), seed + 3)
    return img, sm, tr, dat


def _per_slice(a, b, batched):
    return a[b] if batched else a


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


SHAPES = [
    # nx, ny, nc, nk, batch
    (32, 32, 4, 1024, 1),
    (5, 7, 3, 77, 2),
    (37, 33, 2, 130, 1),
    (64, 48, 9, 200, 3),
    (20, 300, 3, 70, 1),     # two 256-row passes in the forward
    (130, 70, 17, 333, 1),   # three coil groups and ragged tiles in the adjoint
    (1, 1, 1, 1, 1),         # degenerate single pixel / sample
]


PRECS = [mri.FP32, mri.BF16X3, mri.FP16X3]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("nx,ny,nc,nk,batch", SHAPES)
def test_forward_parity(nx, ny, nc, nk, batch, prec):
    img, sm, tr, _ = _inputs(nx, ny, nc, nk, batch, 10)
    got = mri.nudft_forward(_gpu(img), _gpu(sm), _gpu(tr), precision=prec).cpu().numpy()
    ref = np.stack([onudft.forward(img[b], sm, tr) for b in range(batch)])
    assert got.shape == ref.shape
    assert rel(got, ref) <= TOL


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("nx,ny,nc,nk,batch", SHAPES)
def test_adjoint_parity(nx, ny, nc, nk, batch, prec):
    _, sm, tr, dat = _inputs(nx, ny, nc, nk, batch, 20)
    got = mri.nudft_adjoint(_gpu(dat), _gpu(sm), _gpu(tr), ny, nx, precision=prec).cpu().numpy()
    ref = np.stack([onudft.adjoint(dat[b], sm, tr) for b in range(batch)])
    assert rel(got, ref) <= TOL


def test_batched_maps_and_trajectories():
    nx, ny, nc, nk, batch = 24, 20, 3, 150, 3
    img, sm, tr, dat = _inputs(nx, ny, nc, nk, batch, 30, traj_batched=True, smaps_batched=True)
    f = mri.nudft_forward(_gpu(img), _gpu(sm), _gpu(tr)).cpu().numpy()
    a = mri.nudft_adjoint(_gpu(dat), _gpu(sm), _gpu(tr), ny, nx).cpu().numpy()
    for b in range(batch):
        assert rel(f[b], onudft.forward(img[b], sm[b], tr[b])) <= TOL
        assert rel(a[b], onudft.adjoint(dat[b], sm[b], tr[b])) <= TOL


@pytest.mark.parametrize("nx,ny", [(8, 8), (16, 12), (7, 9)])
def test_cartesian_trajectory_matches_oracle_fft_case(nx, ny):
    img = synth.random_complex((1, ny, nx), 40)
    tr = synth.cartesian_trajectory(nx, ny)
    one = np.ones((1, ny, nx), np.complex64)
    got = mri.nudft_forward(_gpu(img), _gpu(one), _gpu(tr)).cpu().numpy()[0, 0]
    ref = onudft.forward(img[0], one, tr)[0]
    assert rel(got, ref) <= TOL


@pytest.mark.parametrize("prec", PRECS)
def test_gpu_adjoint_identity(prec):
    nx, ny, nc, nk = 48, 40, 5, 700
    img, sm, tr, dat = _inputs(nx, ny, nc, nk, 1, 50)
    f = mri.nudft_forward(_gpu(img), _gpu(sm), _gpu(tr), precision=prec).cpu().numpy().astype(np.complex128)
    a = mri.nudft_adjoint(_gpu(dat), _gpu(sm), _gpu(tr), ny, nx, precision=prec).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(f.ravel(), dat.ravel().astype(np.complex128))
    rhs = np.vdot(img.ravel().astype(np.complex128), a.ravel())
    # each side carries the error of one operator: |err| <= tol ||F x|| ||y|| per side
    scale = np.linalg.norm(f) * np.linalg.norm(dat.astype(np.complex128))
    assert abs(lhs - rhs) <= 2 * TOL * scale


@pytest.mark.parametrize("prec", PRECS)
def test_bitwise_reproducible(prec):
    nx, ny, nc, nk = 96, 64, 6, 3000
    img, sm, tr, dat = _inputs(nx, ny, nc, nk, 1, 60)
    g = [_gpu(a) for a in (img, sm, tr, dat)]
    f1 = mri.nudft_forward(g[0], g[1], g[2], precision=prec)
    f2 = mri.nudft_forward(g[0], g[1], g[2], precision=prec)
    a1 = mri.nudft_adjoint(g[3], g[1], g[2], ny, nx, precision=prec)
    a2 = mri.nudft_adjoint(g[3], g[1], g[2], ny, nx, precision=prec)
    assert torch.equal(f1, f2) and torch.equal(a1, a2)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("wl,batch", [(synth.ADMM256, 1), (synth.SLICES384, 2)])
def test_full_size_sampled(wl, batch, prec):
    # Full workload shapes; the oracle recomputes 96 sampled outputs one by one.
    rng = np.random.default_rng(70)
    p = synth.make_problem(wl, batch=batch)
    img = p.truth + synth.random_complex(p.truth.shape, 71) * np.complex64(0.1)
    gi, gs, gt = _gpu(img), _gpu(p.smaps), _gpu(p.traj)
    f = mri.nudft_forward(gi, gs, gt, precision=prec).cpu().numpy()
    dat = synth.random_complex((batch, wl.nc, wl.nk), 72)
    a = mri.nudft_adjoint(_gpu(dat), gs, gt, wl.ny, wl.nx, precision=prec).cpu().numpy()
    for b in range(batch):
        coils = rng.integers(0, wl.nc, 48)
        ks = rng.integers(0, wl.nk, 48)
        ks[:4] = [0, wl.nk - 1, wl.nk // 2, 63]
        ref = onudft.forward_samples(img[b], p.smaps, p.traj, coils, ks)
        assert rel(f[b][coils, ks], ref) <= TOL
        rows = rng.integers(0, wl.ny, 48)
        cols = rng.integers(0, wl.nx, 48)
        rows[:2], cols[:2] = [0, wl.ny - 1], [wl.nx - 1, 0]
        ref = onudft.adjoint_pixels(dat[b], p.smaps, p.traj, rows, cols)
        assert rel(a[b][rows, cols], ref) <= TOL


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("nx,ny,nc,nk", [(2048, 3, 64, 700), (5, 2048, 7, 333)])
def test_maximum_dimensions(nx, ny, nc, nk, prec):
    # MRI_MAX_DIM rows or columns with MRI_MAX_COILS coils: 256 K-steps per
    # forward pass along x, or eight 256-row passes along y; 8 coil groups in
    # the adjoint.
    img, sm, tr, dat = _inputs(nx, ny, nc, nk, 1, 85)
    f = mri.nudft_forward(_gpu(img), _gpu(sm), _gpu(tr), precision=prec).cpu().numpy()[0]
    a = mri.nudft_adjoint(_gpu(dat), _gpu(sm), _gpu(tr), ny, nx, precision=prec).cpu().numpy()[0]
    assert rel(f, onudft.forward(img[0], sm, tr)) <= TOL
    assert rel(a, onudft.adjoint(dat[0], sm, tr)) <= TOL


def test_split_forms_error_ordering():
    # Per-operator error of each form on one mid-size problem.  The bf16 split
    # keeps ~16 bits per operand and its product error dominates; the fp16
    # split keeps ~22, below FP32 accumulation's own rounding, so FP16x3 lands
    # at the FP32 form's error.
    nx, ny, nc, nk = 80, 72, 5, 2500
    img, sm, tr, dat = _inputs(nx, ny, nc, nk, 1, 90)
    fref = onudft.forward(img[0], sm, tr)
    aref = onudft.adjoint(dat[0], sm, tr)
    err = {}
    for prec in PRECS:
        f = mri.nudft_forward(_gpu(img), _gpu(sm), _gpu(tr), precision=prec).cpu().numpy()[0]
        a = mri.nudft_adjoint(_gpu(dat), _gpu(sm), _gpu(tr), ny, nx, precision=prec).cpu().numpy()[0]
        err[prec] = (rel(f, fref), rel(a, aref))
    print("relative error (forward, adjoint):", {mri.PRECISION_NAMES[p]: e for p, e in err.items()})
    for k in range(2):
        assert err[mri.FP16X3][k] <= 1e-6
        assert err[mri.FP16X3][k] * 4 <= err[mri.BF16X3][k]
        assert err[mri.FP16X3][k] <= 2 * err[mri.FP32][k] + 1e-7


@pytest.mark.parametrize("scale", [1e-30, 1e-8, 1e8, 1e30])
def test_fp16x3_extreme_scales(scale):
    # Row and coil scales follow the data: the relative error does not depend
    # on the magnitude of the inputs, down to FP32's small normal numbers and
    # up to its large ones.  Rows of the image also span 12 decades.
    nx, ny, nc, nk = 40, 36, 3, 600
    img, sm, tr, dat = _inputs(nx, ny, nc, nk, 1, 95)
    img = (img * (10.0 ** ((np.arange(ny) % 13) - 6))[None, :, None]).astype(np.complex64)
    img = (img * np.float32(scale)).astype(np.complex64)
    dat = (dat * np.float32(scale)).astype(np.complex64)
    f = mri.nudft_forward(_gpu(img), _gpu(sm), _gpu(tr), precision=mri.FP16X3).cpu().numpy()[0]
    a = mri.nudft_adjoint(_gpu(dat), _gpu(sm), _gpu(tr), ny, nx, precision=mri.FP16X3).cpu().numpy()[0]
    assert np.isfinite(f).all() and np.isfinite(a).all()
    assert rel(f, onudft.forward(img[0], sm, tr)) <= 1e-6
    assert rel(a, onudft.adjoint(dat[0], sm, tr)) <= 1e-6


@pytest.mark.parametrize("prec", PRECS)
def test_zero_and_nonfinite_inputs(prec):
    nx, ny, nc, nk = 24, 20, 2, 300
    img, sm, tr, dat = _inputs(nx, ny, nc, nk, 1, 97)
    z = mri.nudft_forward(_gpu(np.zeros_like(img)), _gpu(sm), _gpu(tr), precision=prec).cpu().numpy()
    za = mri.nudft_adjoint(_gpu(np.zeros_like(dat)), _gpu(sm), _gpu(tr), ny, nx, precision=prec).cpu().numpy()
    assert not z.any() and not za.any()
    # a NaN in the input reaches the output (the solver's status check relies on it)
    img[0, 3, 5] = np.nan
    dat[0, 1, 7] = np.nan
    f = mri.nudft_forward(_gpu(img), _gpu(sm), _gpu(tr), precision=prec).cpu().numpy()
    a = mri.nudft_adjoint(_gpu(dat), _gpu(sm), _gpu(tr), ny, nx, precision=prec).cpu().numpy()
    assert np.isnan(f).any() and np.isnan(a).any()


@pytest.mark.parametrize("prec", PRECS)
def test_full_batch_launch_sampled(prec):
    # The 32-slice 384x384 batch exactly as the batch benchmark launches it
    # (one grouped launch per operator over all slices); the oracle checks
    # sampled outputs of the first, a middle and the last slice.
    wl = synth.SLICES384
    rng = np.random.default_rng(75)
    sm = synth.coil_maps(wl.nx, wl.ny, wl.nc)
    tr = synth.radial_trajectory(wl.n_spokes, wl.n_readout)
    img = synth.random_complex((wl.batch, wl.ny, wl.nx), 76)
    dat = synth.random_complex((wl.batch, wl.nc, wl.nk), 77)
    gs, gt = _gpu(sm), _gpu(tr)
    f = mri.nudft_forward(_gpu(img), gs, gt, precision=prec)
    a = mri.nudft_adjoint(_gpu(dat), gs, gt, wl.ny, wl.nx, precision=prec)
    for b in (0, 17, wl.batch - 1):
        coils = rng.integers(0, wl.nc, 32)
        ks = rng.integers(0, wl.nk, 32)
        got = f[b].cpu().numpy()[coils, ks]
        assert rel(got, onudft.forward_samples(img[b], sm, tr, coils, ks)) <= TOL
        rows = rng.integers(0, wl.ny, 32)
        cols = rng.integers(0, wl.nx, 32)
        got = a[b].cpu().numpy()[rows, cols]
        assert rel(got, onudft.adjoint_pixels(dat[b], sm, tr, rows, cols)) <= TOL


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("traj_batched", [False, True])
def test_adjoint_plan_matches_single_calls(prec, traj_batched):
    # Phase tables built once (nudft_adjoint_prepare) and reused by several
    # prepared calls give the single-call results bit for bit, and stay
    # within the per-operator bar of the oracle.
    nx, ny, nc, nk, batch = 70, 46, 5, 900, 2
    img, sm, tr, _ = _inputs(nx, ny, nc, nk, batch, 110, traj_batched=traj_batched)
    gs, gt = _gpu(sm), _gpu(tr)
    plan = mri.AdjointPlan(gs, gt, ny, nx, batch=batch, precision=prec)
    for seed in (111, 112):
        dat = synth.random_complex((batch, nc, nk), seed)
        got = plan(_gpu(dat))
        ref = mri.nudft_adjoint(_gpu(dat), gs, gt, ny, nx, precision=prec)
        assert torch.equal(got, ref)
        g = got.cpu().numpy()
        for b in range(batch):
            assert rel(g[b], onudft.adjoint(dat[b], sm, _per_slice(tr, b, traj_batched))) <= TOL


@pytest.mark.parametrize("nx,ny,batch", [(32, 32, 1), (7, 5, 3), (1, 9, 2), (300, 2, 1)])
def test_tv_parity(nx, ny, batch):
    x = synth.random_complex((batch, ny, nx), 80)
    g = synth.random_complex((batch, 2, ny, nx), 81)
    gf = mri.tv_forward(_gpu(x)).cpu().numpy()
    ga = mri.tv_adjoint(_gpu(g)).cpu().numpy()
    for b in range(batch):
        np.testing.assert_allclose(gf[b], otv.tv_forward(x[b]), rtol=0, atol=1e-6)
        np.testing.assert_allclose(ga[b], otv.tv_adjoint(g[b]), rtol=0, atol=1e-6)
