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
  least-squares problem whose iterates move by several 1e-3 (image NRMSE)
  under any FP32-sized rounding: the oracle itself, with only its operator
  outputs rounded to complex64 or carrying relative errors of 1e-7 .. 1e-6,
  moves that far from its FP64 run (tests/golden/tolerances.json).  So the
  image is held to twice the largest of those shifts (tests/bars.py), not
  the 1e-4 of the benchmark settings, and its error against the phantom must
  equal the oracle's to 1 %;
* the large-image case of Sec. VI (1024 x 512, 12 coils, 101 x 1024 samples,
  Table I settings) at 1 ADMM x 2 CG against a stored oracle reconstruction,
  and the full Table I run against properties.
"""
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
    assert e <= bars.TABLE1_128x64
    assert abs(e_truth - e_truth_ref) <= 0.01 * e_truth_ref


GOLDEN_LARGE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_large_oracle.npz")


@pytest.mark.parametrize("prec", [mri.FP32, mri.FP16X3, mri.BF16X3])
def test_table1_large_image_reduced_counts_against_stored_oracle(prec):
    # 1024x512 / 12 coils / 101x1024 samples with the Table I lambda, beta and
    # tolerances at 1 ADMM x 2 CG, on the data stored with the oracle's own
    # reconstruction (tests/golden/make_table1_large_golden.py): FP32 and
    # FP16x3 within the 1e-4 bar, BF16x3 within its bar derived from the
    # oracle's sensitivity at these counts (tests/bars.py).
    wl = synth.TABLE1_1024x512
    g = np.load(GOLDEN_LARGE)
    na, ncg = int(g["admm_max"]), int(g["cg_max"])
    p = synth.make_problem(wl, batch=1)
    img, st = mri.admm_solve(_gpu(p.smaps), _gpu(p.traj), _gpu(g["data"][None]), wl.ny, wl.nx,
                             mri.AdmmParams(wl.lam, wl.beta, na, ncg, rtol=wl.rtol, atol=wl.atol, precision=prec))
    assert st[0]["status"] == 0
    assert st[0]["admm_iters"] == int(g["admm_iters"]) and st[0]["cg_steps"] == int(g["cg_steps"])
    e = _rel(img.cpu().numpy()[0], g["image"])
    print(f"{mri.PRECISION_NAMES[prec]}: 1024x512 Table I {na}x{ncg} image NRMSE vs stored oracle {e:.3e}")
    assert e <= (1e-4 if prec != mri.BF16X3 else bars.BF16X3_TABLE1_LARGE)


def test_table1_parameters_large_image():
    # The 1024x512 / 12-coil / 101x1024-sample problem of Sec. VI with the
    # full Table I settings (up to 5 ADMM x 20 CG).  The oracle's run at these
    # counts would take hours, so the solve is held to properties: the
    # device's stopping rules give valid counts; the data residual
    # ||F x - d|| / ||d|| falls well below that of the oracle's 1 x 2 run
    # (stored golden) and under 1e-3 (measured 3.1e-4); and the two forms with
    # FP32-level operators (FP32, FP16x3) reach the same image to the
    # ill-conditioning bound derived at 128x64, with the same error against
    # the phantom to 1 %.  (Its operators are checked against the oracle on
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
        assert resid <= 1e-3 and resid < float(np.load(GOLDEN_LARGE)["resid"])
        out[prec] = (img.cpu().numpy()[0], e_truth)
    (a, ea), (b, eb) = out[mri.FP32], out[mri.FP16X3]
    assert _rel(b, a) <= bars.TABLE1_128x64
    assert abs(ea - eb) <= 0.01 * ea
