"""GPU parity of admm_solve (Alg. 4 with CG of Alg. 2) against the FP64
oracle, through the C ABI.  Bar: final-image NRMSE <= 1e-4."""
import os

import numpy as np
import pytest
import torch

import bars
from oracle import admm as oadmm
from oracle import nudft as onudft
from paper_2006_14080_amd import mri, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"
NRMSE = 1e-4


def nrmse(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _data(p):
    """k-space data of each slice: oracle F(truth) + noise, rounded to complex64."""
    return np.stack([onudft.forward(p.truth[b], p.smaps, p.traj) + p.noise[b]
                     for b in range(p.truth.shape[0])]).astype(np.complex64)


def _solve(p, data, params, x0=None):
    wl = p.wl
    img, st = mri.admm_solve(_gpu(p.smaps), _gpu(p.traj), _gpu(data), wl.ny, wl.nx, params,
                             x0=None if x0 is None else _gpu(x0))
    return img.cpu().numpy(), st


def _oracle(p, data, b, lam, beta, na, nc, **kw):
    return oadmm.admm(data[b], p.smaps, p.traj, lam, beta, na, nc, **kw)


# BF16x3 keeps ~16 bits per operand (per-operator error ~4e-6).  The oracle's
# own 10 x 3 solve at 32x32 moves its image by up to 2.9e-4 when its operators
# carry that error (tests/golden/tolerances.json), so BF16x3 is held to twice
# that there (tests/bars.py); FP32 and FP16x3 (operator errors <= 6e-7, image
# shifts <= 7e-5) meet the 1e-4 bar.
BAR = {mri.FP32: NRMSE, mri.FP16X3: NRMSE, mri.BF16X3: bars.BF16X3_ADMM32}


@pytest.mark.parametrize("prec", [mri.FP32, mri.BF16X3, mri.FP16X3])
def test_admm32_full_counts(prec):
    # The plain 32x32 workload (10 ADMM x 3 CG) in each precision form.
    wl = synth.ADMM32
    p = synth.make_problem(wl)
    data = _data(p)
    img, st = _solve(p, data, mri.AdmmParams(wl.lam, wl.beta, wl.admm_iters, wl.cg_iters, precision=prec))
    ref = _oracle(p, data, 0, wl.lam, wl.beta, wl.admm_iters, wl.cg_iters)
    assert st[0]["status"] == 0
    assert st[0]["admm_iters"] == ref.admm_iters and st[0]["cg_steps"] == ref.cg_steps
    e = nrmse(img[0], ref.image)
    print(f"{mri.PRECISION_NAMES[prec]}: 32x32 10x3 image NRMSE vs oracle {e:.3e}")
    assert e <= BAR[prec]


@pytest.mark.parametrize("warm", [True, False])
def test_small_ragged_problem_with_x0(warm):
    wl = synth.Workload("t", 20, 13, 3, 7, 43, 2e-3, 0.7, 4, 3, seed=9)
    p = synth.make_problem(wl)
    data = _data(p)
    x0 = (p.truth * np.complex64(0.5 + 0.25j)).astype(np.complex64)
    img, st = _solve(p, data, mri.AdmmParams(wl.lam, wl.beta, 4, 3, cg_warm_start=warm), x0=x0)
    ref = _oracle(p, data, 0, wl.lam, wl.beta, 4, 3, x0=x0[0], warm=warm)
    assert nrmse(img[0], ref.image) <= NRMSE
    assert st[0]["cg_steps"] == ref.cg_steps


def test_batch_is_independent_slices_bitwise():
    wl = synth.Workload("t", 24, 24, 3, 8, 48, 1e-3, 1.0, 3, 2, batch=3, seed=30)
    p = synth.make_problem(wl)
    data = _data(p)
    prm = mri.AdmmParams(wl.lam, wl.beta, 3, 2)
    img, _ = _solve(p, data, prm)
    for b in range(3):
        q = synth.Problem(wl, p.truth[b:b + 1], p.smaps, p.traj, p.noise[b:b + 1])
        one, _ = _solve(q, data[b:b + 1], prm)
        assert np.array_equal(one[0], img[b])
        ref = _oracle(p, data, b, wl.lam, wl.beta, 3, 2)
        assert nrmse(img[b], ref.image) <= NRMSE


@pytest.mark.parametrize("prec", [mri.FP32, mri.FP16X3])
def test_batch_with_per_slice_trajectories_and_maps(prec):
    # Each slice has its own trajectory (random points) and coil maps, so the
    # solve builds one set of adjoint phase tables per slice; every slice of
    # the batched solve equals its solo solve bit for bit and the oracle.
    nx, ny, nc, nk, nb = 20, 28, 3, 400, 3
    truth = np.stack([synth.ellipse_phantom(nx, ny, 40 + b) for b in range(nb)])
    maps = np.stack([synth.random_complex((nc, ny, nx), 50 + b) * np.complex64(0.3) + synth.coil_maps(nx, ny, nc)
                     for b in range(nb)]).astype(np.complex64)
    traj = np.stack([synth.random_trajectory(nk, 60 + b) for b in range(nb)])
    data = np.stack([onudft.forward(truth[b], maps[b], traj[b]) + synth.complex_noise((nc, nk), 1e-3, 70 + b)
                     for b in range(nb)]).astype(np.complex64)
    prm = mri.AdmmParams(1e-3, 1.0, 3, 2, precision=prec)
    img, st = mri.admm_solve(_gpu(maps), _gpu(traj), _gpu(data), ny, nx, prm)
    img = img.cpu().numpy()
    for b in range(nb):
        assert st[b]["status"] == 0
        one, _ = mri.admm_solve(_gpu(maps[b]), _gpu(traj[b]), _gpu(data[b:b + 1]), ny, nx, prm)
        assert np.array_equal(one.cpu().numpy()[0], img[b])
        ref = oadmm.admm(data[b], maps[b], traj[b], 1e-3, 1.0, 3, 2)
        assert nrmse(img[b], ref.image) <= NRMSE


def test_zero_data_stops_after_one_iteration():
    wl = synth.Workload("t", 16, 16, 2, 4, 32, 1e-3, 1.0, 5, 4, seed=3)
    p = synth.make_problem(wl)
    data = np.zeros((1, wl.nc, wl.nk), np.complex64)
    img, st = _solve(p, data, mri.AdmmParams(wl.lam, wl.beta, 5, 4))
    assert st[0]["admm_iters"] == 1 and st[0]["cg_steps"] == 0 and st[0]["status"] == 0
    assert np.all(img == 0)


def test_tolerances_stop_on_device():
    wl = synth.Workload("t", 24, 20, 3, 10, 48, 1e-7, 1.0, 5, 20, seed=12)
    p = synth.make_problem(wl)
    data = _data(p)
    # atol^2 ~ 1e5: the first CG solve stops after 7 steps (tau 2.1e5 -> 5.7e4),
    # the second starts below atol^2 and takes no step, so alpha = 0 ends ADMM.
    prm = mri.AdmmParams(wl.lam, wl.beta, 5, 20, rtol=0.3, atol=316.0)
    img, st = _solve(p, data, prm)
    ref = _oracle(p, data, 0, wl.lam, wl.beta, 5, 20, rtol=0.3, atol=316.0)
    assert ref.admm_iters == 2 and ref.cg_steps == 7
    assert st[0]["admm_iters"] == ref.admm_iters < 5
    assert st[0]["cg_steps"] == ref.cg_steps < 5 * 20
    assert nrmse(img[0], ref.image) <= NRMSE


@pytest.mark.parametrize("prec", [mri.FP32, mri.BF16X3, mri.FP16X3])
def test_admm256_shape_reduced_counts(prec):
    # The 256x256, 8-coil, 64x512-sample launch configuration of the benchmark,
    # with 2 ADMM x 2 CG steps so the oracle finishes in seconds.
    wl = synth.ADMM256
    p = synth.make_problem(wl)
    data = _data(p)
    img, st = _solve(p, data, mri.AdmmParams(wl.lam, wl.beta, 2, 2, precision=prec))
    ref = _oracle(p, data, 0, wl.lam, wl.beta, 2, 2)
    assert st[0]["admm_iters"] == 2 and st[0]["cg_steps"] == 4
    assert nrmse(img[0], ref.image) <= NRMSE


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "admm256_oracle.npz")


def _admm256_full(prec):
    # The whole benchmark solve (256x256, 8 coils, 64x512 samples, 30 ADMM x
    # 5 CG) on the data stored with the oracle's own 30 x 5 reconstruction
    # (tests/golden/make_admm256_golden.py; the oracle takes minutes here).
    wl = synth.ADMM256
    g = np.load(GOLDEN)
    p = synth.make_problem(wl)
    img, st = _solve(p, g["data"][None], mri.AdmmParams(wl.lam, wl.beta, wl.admm_iters, wl.cg_iters,
                                                        precision=prec))
    assert st[0]["status"] == 0
    assert st[0]["admm_iters"] == int(g["admm_iters"]) == 30
    assert st[0]["cg_steps"] == int(g["cg_steps"]) == 150
    e = nrmse(img[0], g["image"])
    print(f"{mri.PRECISION_NAMES[prec]}: image NRMSE vs stored oracle = {e:.3e}")
    return e


@pytest.mark.parametrize("prec", [mri.FP32, mri.FP16X3])
def test_admm256_full_counts_against_stored_oracle(prec):
    assert _admm256_full(prec) <= NRMSE


def test_admm256_full_counts_bf16x3():
    # The bf16 split keeps ~16 bits per operand (per-operator error ~4e-6),
    # and 150 CG steps amplify operator errors, so which image BF16x3 reaches
    # depends on rounding order.  Its bar is derived from the oracle: twice
    # the largest shift of the oracle's own 30 x 5 image when its operators
    # carry BF16x3's error (tests/bars.py, tests/golden/tolerances.json).
    assert _admm256_full(mri.BF16X3) <= bars.BF16X3_ADMM256


GOLDEN_384 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "slices384_oracle.npz")


@pytest.mark.parametrize("prec", [mri.FP32, mri.FP16X3, mri.BF16X3])
def test_slices384_batch_solve_against_stored_oracle(prec):
    # The 32-slice 384x384 batch (16 coils, 128 x 768 samples, lambda 5e-4) as
    # one batched solve, so every operator is one grouped launch over all 32
    # slices, at 2 ADMM x 2 CG.  Slices 0 and 31 solve the data stored with the
    # oracle's reconstructions of them (tests/golden/make_slices384_golden.py);
    # the other 30 take the GPU forward of their phantoms plus their noise.
    # FP32 and FP16x3 within the 1e-4 bar; BF16x3 within its bar derived from
    # the oracle's sensitivity on this slice at these counts (tests/bars.py).
    wl = synth.SLICES384
    g = np.load(GOLDEN_384)
    na, ncg = int(g["admm_iters"]), int(g["cg_iters"])
    smaps = synth.coil_maps(wl.nx, wl.ny, wl.nc)
    traj = synth.radial_trajectory(wl.n_spokes, wl.n_readout)
    sm, tr = _gpu(smaps), _gpu(traj)
    truth = _gpu(np.stack([synth.slice_phantom(wl, b) for b in range(wl.batch)]))
    data = mri.nudft_forward(truth, sm, tr, precision=mri.FP32)
    for b in range(wl.batch):
        data[b] += _gpu(synth.slice_noise(wl, b).astype(np.complex64))
    for i, b in enumerate(g["slices"]):
        data[int(b)] = _gpu(g["data"][i])
    img, st = mri.admm_solve(sm, tr, data, wl.ny, wl.nx,
                             mri.AdmmParams(wl.lam, wl.beta, na, ncg, precision=prec))
    img = img.cpu().numpy()
    for i, b in enumerate(g["slices"]):
        b = int(b)
        assert st[b]["status"] == 0
        assert (st[b]["admm_iters"], st[b]["cg_steps"]) == tuple(int(v) for v in g["counts"][i])
        e = nrmse(img[b], g["images"][i])
        print(f"{mri.PRECISION_NAMES[prec]}: 32x384^2 batch, slice {b}, {na}x{ncg}: image NRMSE vs stored "
              f"oracle {e:.3e}")
        assert e <= (NRMSE if prec != mri.BF16X3 else bars.BF16X3_SLICES384)


def _nufft_oracle_admm(data, smaps, traj, ny, nx, lam, beta, na, ncg):
    """The oracle's ADMM with F applied by the oracle NUFFT (width 6,
    oversampling 2): the reference of admm_solve's MRI_NUFFT mode."""
    from oracle import nufft as onufft
    from oracle import tv as otv
    plan = onufft.Plan(nx, ny, traj, width=6, sigma=2.0)

    def apply_a(v):
        return onufft.adjoint(onufft.forward(v, smaps, plan), smaps, plan) + \
            0.5 * beta * otv.tv_adjoint(otv.tv_forward(v))

    return oadmm.admm(data, smaps, traj, lam, beta, na, ncg, apply_a=apply_a,
                      adjoint=lambda u: onufft.adjoint(u, smaps, plan))


@pytest.mark.parametrize("wl,na,ncg", [(synth.ADMM32, 10, 3), (synth.ADMM256, 2, 2)])
def test_nufft_operator_solve(wl, na, ncg):
    # admm_solve with the NUFFT operator against the oracle ADMM on the oracle
    # NUFFT (1e-4 bar), and how far it lands from the dense-operator oracle
    # solve (the operator's approximation, reported).
    p = synth.make_problem(wl)
    data = _data(p)
    img, st = _solve(p, data, mri.AdmmParams(wl.lam, wl.beta, na, ncg, precision=mri.NUFFT))
    ref = _nufft_oracle_admm(data[0], p.smaps, p.traj, wl.ny, wl.nx, wl.lam, wl.beta, na, ncg)
    assert st[0]["status"] == 0 and st[0]["admm_iters"] == ref.admm_iters and st[0]["cg_steps"] == ref.cg_steps
    e = nrmse(img[0], ref.image)
    dense = _oracle(p, data, 0, wl.lam, wl.beta, na, ncg).image
    print(f"nufft solve {wl.name} {na}x{ncg}: NRMSE vs oracle NUFFT solve {e:.3e}, vs dense oracle solve "
          f"{nrmse(img[0], dense):.3e}")
    assert e <= NRMSE


def test_nufft_mode_rejected_where_unsupported():
    from paper_2006_14080_amd import serve
    with pytest.raises(mri.MriError):
        serve.Server(1 << 26, max_slots=2, precision=mri.NUFFT)
    wl = synth.ADMM32
    p = synth.make_problem(wl)
    with pytest.raises(mri.MriError):
        mri.nudft_forward(_gpu(p.truth), _gpu(p.smaps), _gpu(p.traj), precision=mri.NUFFT)
