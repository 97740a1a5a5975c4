"""The C ABI library loads, exports every entry point include/mri_admm.h
declares, agrees with the binding on struct layouts, and rejects bad
arguments on the host before touching the GPU (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_2006_14080_amd import mri

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mri_admm.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mri.LIB_PATH):
        pytest.fail("libmriadmm.so has not been built (run python -m paper_2006_14080_amd.build)")
    return mri.load()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ["nudft_forward", "nudft_adjoint", "nudft_adjoint_prepare", "nudft_adjoint_prepared",
              "tv_forward", "tv_adjoint", "admm_solve", "mri_workspace_bytes", "mri_strerror"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_struct_layouts():
    assert ctypes.sizeof(mri.MriShape) == 40
    assert mri.MriShape.nk.offset == 16
    assert ctypes.sizeof(mri.MriAdmmParams) == 48
    assert ctypes.sizeof(mri.MriAdmmStats) == 32


def test_adjoint_split(lib):
    # 256^2 / 8 coils / 32768 samples: 16 ranges of 2048 samples, one coil
    # group, so 16 partial images; 384^2 / 16 coils / 98304 samples: two coil
    # groups of 8.
    assert mri.adjoint_split(mri.make_shape(256, 256, 8, 32768)) == {"ksplit": 16, "kper": 2048, "planes": 16}
    s384 = mri.adjoint_split(mri.make_shape(384, 384, 16, 98304, batch=32))
    assert s384["planes"] == 2 * s384["ksplit"] and s384["ksplit"] * s384["kper"] >= 98304
    # fewer samples than one range of 256: a single range
    assert mri.adjoint_split(mri.make_shape(384, 384, 1, 64))["planes"] == 1
    assert lib.mri_adjoint_split(ctypes.byref(mri.make_shape(0, 8, 1, 8)), None, None, None) == -1


def _workgroups(nx, ny, sp):
    # 128 x 32 pixel tiles x (coil group, sample range) partial images
    return -(-nx // 128) * -(-ny // 32) * sp["planes"]


@pytest.mark.parametrize("nx,ny,nc,nk,ksplit", [
    (256, 256, 8, 32768, 16),      # 256 workgroups, one round of the 256 CUs
    (384, 384, 32, 98304, 5),      # 720 workgroups in three rounds (94 %); 8 ranges left a round near empty
    (384, 384, 16, 98304, 7),      # 504 workgroups (98 %)
    (128, 128, 32, 32768, 16),     # 4 coil groups x 4 tiles x 16 ranges
    (1024, 512, 12, 103424, 2),    # at most 65536 samples per range
    (256, 256, 8, 4096, 16),       # one GPU's share of an 8-way k-space split
])
def test_adjoint_split_fills_the_cus(nx, ny, nc, nk, ksplit):
    sp = mri.adjoint_split(mri.make_shape(nx, ny, nc, nk))
    assert sp["ksplit"] == ksplit
    assert 256 <= sp["kper"] <= 65536 and sp["kper"] % 8 == 0
    assert sp["ksplit"] * sp["kper"] >= nk > (sp["ksplit"] - 1) * sp["kper"]
    w = _workgroups(nx, ny, sp)
    assert w >= 256 and w / (-(-w // 256) * 256) >= 0.9


def test_adjoint_split_of_small_problems_takes_the_most_ranges():
    # a problem that cannot fill one round of the CUs: as many ranges as the
    # 256-sample minimum allows
    sp = mri.adjoint_split(mri.make_shape(128, 128, 4, 8192))
    assert sp["ksplit"] == 8192 // 256 and _workgroups(128, 128, sp) < 256


def test_strerror(lib):
    assert lib.mri_strerror(0) == b"success"
    assert b"invalid" in lib.mri_strerror(-1)
    assert b"unknown" in lib.mri_strerror(12345)


def test_workspace_sizes(lib):
    sh = mri.make_shape(256, 256, 8, 32768)
    p = mri.AdmmParams(1e-3, 1.0, 30, 5).c()
    # forward: the coil-weighted image, rows padded to a multiple of 8; the
    # split forms keep it pre-split (16-bit hi and lo of re and im: 8 B per
    # element, as in FP32), FP16x3 with one float scale per row
    assert mri.workspace_bytes(sh, mri.OP_FORWARD) == 8 * 256 * 256 * 8 + 4 * 8 * 256
    adj = mri.workspace_bytes(sh, mri.OP_ADJOINT)
    # partial images plus the phase tables exp(+i w x), exp(+i w y): (nx + ny) nk
    assert adj >= 256 * 256 * 8 + (256 + 256) * 32768 * 8 and adj % 256 == 0
    # per-slice trajectories: one table per slice
    shb = mri.make_shape(256, 256, 8, 32768, batch=3, traj_batched=True)
    assert mri.workspace_bytes(shb, mri.OP_ADJOINT) >= 3 * (256 + 256) * 32768 * 8
    total = mri.workspace_bytes(sh, mri.OP_ADMM, p)
    assert total > 12 * 256 * 256 * 8 + 8 * 32768 * 8
    bad = mri.make_shape(0, 256, 8, 32768)
    assert mri.workspace_bytes(bad, mri.OP_ADMM, p) == 0


@pytest.mark.parametrize("field,value", [("nx", 0), ("ny", -1), ("ncoils", 0), ("nk", 0),
                                         ("batch", 0), ("traj_batched", 2), ("nx", 4096)])
def test_bad_shapes_rejected_on_host(lib, field, value):
    sh = mri.make_shape(8, 8, 2, 16)
    setattr(sh, field, value)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    rc = lib.nudft_forward(ctypes.byref(sh), fake, fake, fake, fake, 0, None, 0, None)
    assert rc == -1


def test_bad_params_rejected_on_host(lib):
    sh = mri.make_shape(8, 8, 2, 16)
    fake = ctypes.c_void_p(0x1000)
    for kw in [dict(lam=-1.0), dict(beta=0.0), dict(admm_iters=-1), dict(cg_iters=-2),
               dict(rtol=-1e-3), dict(precision=7)]:
        args = dict(lam=1e-3, beta=1.0, admm_iters=2, cg_iters=2)
        args.update(kw)
        p = mri.AdmmParams(**args).c()
        rc = lib.admm_solve(ctypes.byref(sh), fake, fake, fake, None, ctypes.byref(p), fake, None,
                            fake, 1 << 30, None)
        assert rc == -1, kw
    p = mri.AdmmParams(1e-3, 1.0, 2, 2).c()
    rc = lib.admm_solve(ctypes.byref(sh), fake, fake, fake, None, ctypes.byref(p), fake, None, fake, 16, None)
    assert rc == -2   # workspace too small


def test_null_pointers_rejected(lib):
    sh = mri.make_shape(8, 8, 2, 16)
    fake = ctypes.c_void_p(0x1000)
    assert lib.nudft_forward(ctypes.byref(sh), None, fake, fake, fake, 0, None, 0, None) == -1
    assert lib.tv_forward(ctypes.byref(sh), None, fake, None) == -1
    assert lib.nudft_adjoint(ctypes.byref(sh), fake, fake, fake, fake, 0, None, 0, None) == -2
    n = mri.workspace_bytes(sh, mri.OP_ADJOINT)
    assert lib.nudft_adjoint_prepare(ctypes.byref(sh), None, fake, n, None) == -1
    assert lib.nudft_adjoint_prepare(ctypes.byref(sh), fake, fake, n - 1, None) == -2
    assert lib.nudft_adjoint_prepared(ctypes.byref(sh), fake, fake, fake, None, 0, fake, n, None) == -1
    assert lib.nudft_adjoint_prepared(ctypes.byref(sh), fake, fake, fake, fake, 0, None, 0, None) == -2
    assert lib.nudft_adjoint_prepared(ctypes.byref(sh), fake, fake, fake, fake, 7, fake, n, None) == -1
