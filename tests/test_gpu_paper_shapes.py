"""Paper-shaped stand-ins of Sec. V on the GPU, through the C ABI.

* "inverse DFT" of fully sampled radial data (the adjoint with the conjugate
  coil combine, Alg. 3) on a 128 x 64 grid with 12 coils and 101 spokes x 128
  samples: the paper compares its TPU result with an FP64 CPU result inside
  the phantom (about 0.1 % there); here every precision form is compared with
  the FP64 oracle inside the phantom support and must stay under the 1e-5
  per-operator bar;
* ADMM with the Table I parameters (lambda 1e-7, beta 1, relative tolerance
  1e-4 over at most 5 iterations, CG absolute tolerance 1e-6 over at most 20
  steps) on the x8-undersampled set (13 spokes x 128 samples): the device's
  stopping decisions reproduce the oracle's iteration counts.  With lambda
  this small the 20-step CG solves an almost unregularised, ill-conditioned
  least-squares problem whose iterates move by ~3.5e-3 (image NRMSE) under any
  FP32-sized rounding: the oracle itself, with only its operator outputs
  rounded to complex64, lands 3.2e-3 from its FP64 run, and relative operator
  noise of 1e-7 .. 1e-6 gives 3.6e-3 .. 4.4e-3.  So the image is held to 1e-2
  of the FP64 oracle here (not the 1e-4 of the benchmark settings, which
  FP32 meets at 4.6e-5), and its error against the phantom must equal the
  oracle's to 1 %.
"""
import numpy as np
import pytest
import torch

from oracle import admm as oadmm
from oracle import nudft as onudft
from paper_2006_14080_amd import mri, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _rel(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("prec", [mri.FP32, mri.BF16X3, mri.FP16X3])
def test_inverse_dft_fully_sampled_inside_phantom(prec):
    wl = synth.INVDFT128x64
    p = synth.make_problem(wl)
    data = (onudft.forward(p.truth[0], p.smaps, p.traj) + p.noise[0]).astype(np.complex64)
    ref = onudft.adjoint(data, p.smaps, p.traj)
    got = mri.nudft_adjoint(_gpu(data[None]), _gpu(p.smaps), _gpu(p.traj), wl.ny, wl.nx,
                            precision=prec).cpu().numpy()[0]
    inside = np.abs(p.truth[0]) > 0
    assert inside.sum() > 0.2 * inside.size
    assert _rel(got[inside], ref[inside]) <= 1e-5
    assert _rel(got, ref) <= 1e-5


@pytest.mark.parametrize("prec", [mri.FP32, mri.FP16X3])
def test_table1_parameters_paper_shape(prec):
    wl = synth.TABLE1_128x64
    p = synth.make_problem(wl)
    data = (onudft.forward(p.truth[0], p.smaps, p.traj) + p.noise[0]).astype(np.complex64)
    ref = oadmm.admm(data, p.smaps, p.traj, wl.lam, wl.beta, wl.admm_iters, wl.cg_iters,
                     rtol=wl.rtol, atol=wl.atol)
    img, st = mri.admm_solve(_gpu(p.smaps), _gpu(p.traj), _gpu(data[None]), wl.ny, wl.nx,
                             mri.AdmmParams(wl.lam, wl.beta, wl.admm_iters, wl.cg_iters,
                                            rtol=wl.rtol, atol=wl.atol, precision=prec))
    assert st[0]["status"] == 0
    assert st[0]["admm_iters"] == ref.admm_iters
    assert st[0]["cg_steps"] == ref.cg_steps
    got = img.cpu().numpy()[0]
    e = _rel(got, ref.image)
    e_truth, e_truth_ref = _rel(got, p.truth[0]), _rel(ref.image, p.truth[0])
    print(f"{mri.PRECISION_NAMES[prec]}: Table I run {ref.admm_iters} ADMM / {ref.cg_steps} CG, "
          f"image NRMSE vs oracle {e:.3e}, vs phantom {e_truth:.5f} (oracle {e_truth_ref:.5f})")
    assert e <= 1e-2
    assert abs(e_truth - e_truth_ref) <= 0.01 * e_truth_ref


def test_table1_parameters_large_image():
    # The 1024x512 / 12-coil / 101x1024-sample problem of Sec. VI with the
    # Table I settings.  Each operator here costs 5.2e12 flop, beyond what the
    # FP64 oracle runs in test time, so the solve is held to properties that
    # hold at any size: the device's stopping rules give valid counts and a
    # CG-reduced data residual, and the two forms with FP32-level operators
    # (FP32, FP16x3) reach the same image to the ill-conditioning bound shown
    # against the oracle at 128x64 (1e-2), with the same error against the
    # phantom to 1 %.  (Its operators are checked against the oracle on
    # sampled outputs in test_gpu_shards.py.)
    wl = synth.TABLE1_1024x512
    p = synth.make_problem(wl)
    sm, tr, truth = _gpu(p.smaps), _gpu(p.traj), _gpu(p.truth)
    data = mri.nudft_forward(truth, sm, tr, precision=mri.FP32) + _gpu(p.noise.astype(np.complex64))
    out = {}
    for prec in (mri.FP32, mri.FP16X3):
        img, st = mri.admm_solve(sm, tr, data, wl.ny, wl.nx,
                                 mri.AdmmParams(wl.lam, wl.beta, wl.admm_iters, wl.cg_iters,
                                                rtol=wl.rtol, atol=wl.atol, precision=prec))
        s = st[0]
        assert s["status"] == 0
        assert 1 <= s["admm_iters"] <= wl.admm_iters
        assert 0 <= s["cg_steps"] <= wl.cg_iters * s["admm_iters"]
        resid = float(torch.linalg.vector_norm(mri.nudft_forward(img, sm, tr) - data) /
                      torch.linalg.vector_norm(data))
        e_truth = _rel(img.cpu().numpy()[0], p.truth[0])
        print(f"{mri.PRECISION_NAMES[prec]}: {s['admm_iters']} ADMM / {s['cg_steps']} CG, "
              f"data residual {resid:.4e}, NRMSE vs phantom {e_truth:.5f}")
        assert resid <= 0.5
        out[prec] = (img.cpu().numpy()[0], e_truth)
    (a, ea), (b, eb) = out[mri.FP32], out[mri.FP16X3]
    assert _rel(b, a) <= 1e-2
    assert abs(ea - eb) <= 0.01 * ea
