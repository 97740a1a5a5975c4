"""The Python binding checks every tensor against the shape it passes to the
library, before any library call: a tensor smaller than the shape says would
make the kernels read or write outside it.  CPU tensors reach the shape check
(it runs before the device check), so nothing here launches anything."""
import pytest
import torch

from paper_2006_14080_amd import mri

NX, NY, NC, NK, B = 12, 10, 3, 40, 2
C64, F64 = torch.complex64, torch.float64


def t(*shape, dtype=C64):
    return torch.zeros(shape, dtype=dtype)


@pytest.fixture(scope="module", autouse=True)
def lib():
    return mri.load()


def test_forward_rejects_mismatched_tensors():
    img, sm, tr = t(B, NY, NX), t(NC, NY, NX), t(NK, 2, dtype=F64)
    with pytest.raises(ValueError):
        mri.nudft_forward(t(NY, NX), sm, tr)                         # image not [B, ny, nx]
    with pytest.raises(ValueError):
        mri.nudft_forward(img, t(NC, NY, NX + 1), tr)                # maps on another grid
    with pytest.raises(ValueError):
        mri.nudft_forward(img, sm, t(NK, 3, dtype=F64))              # trajectory not [nk, 2]
    with pytest.raises(ValueError):
        mri.nudft_forward(img, t(B + 1, NC, NY, NX), tr)             # batched maps, wrong batch
    with pytest.raises(ValueError):
        mri.nudft_forward(img, sm, tr, out=t(B, NC, NK - 1))         # output too small
    with pytest.raises(TypeError):
        mri.nudft_forward(img, sm, tr)                               # right shapes, not on the GPU


def test_adjoint_rejects_mismatched_tensors():
    sm, tr = t(NC, NY, NX), t(NK, 2, dtype=F64)
    with pytest.raises(ValueError):
        mri.nudft_adjoint(t(B, NC, NK + 1), sm, tr, NY, NX)          # data longer than traj
    with pytest.raises(ValueError):
        mri.nudft_adjoint(t(B, NC + 1, NK), sm, tr, NY, NX)          # more coils than maps
    with pytest.raises(ValueError):
        mri.nudft_adjoint(t(NC, NK), sm, tr, NY, NX)                 # data not [B, nc, nk]
    with pytest.raises(ValueError):
        mri.nudft_adjoint(t(B, NC, NK), sm, tr, NY, NX, out=t(B, NY, NX - 1))
    with pytest.raises(ValueError):
        mri.nudft_adjoint(t(B, NC, NK), sm, t(B + 1, NK, 2, dtype=F64), NY, NX)
    with pytest.raises(TypeError):
        mri.nudft_adjoint(t(B, NC, NK), sm, tr, NY, NX)


def test_tv_rejects_bad_ranks():
    with pytest.raises(ValueError):
        mri.tv_forward(t(NY, NX))
    with pytest.raises(ValueError):
        mri.tv_adjoint(t(B, 3, NY, NX))


def test_solver_rejects_tensors_that_do_not_match_its_shape():
    sh = mri.make_shape(NX, NY, NC, NK, B)
    solver = mri.AdmmSolver(sh, mri.AdmmParams(1e-3, 1.0, 2, 2), device="cpu")
    sm, tr, d = t(NC, NY, NX), t(NK, 2, dtype=F64), t(B, NC, NK)
    bad = [
        dict(smaps=t(NC - 1, NY, NX)),
        dict(smaps=t(B, NC, NY, NX)),             # batched maps for a shared-map shape
        dict(traj=t(NK - 8, 2, dtype=F64)),
        dict(traj=t(NK, 2)),                      # wrong dtype -> TypeError, checked below
        dict(data=t(B, NC, NK // 2)),
        dict(data=t(B - 1, NC, NK)),
        dict(x0=t(B, NY - 1, NX)),
        dict(out=t(B, NY, NX // 2)),
    ]
    for kw in bad:
        args = dict(smaps=sm, traj=tr, data=d)
        args.update(kw)
        exc = TypeError if "traj" in kw and kw["traj"].dtype != F64 else ValueError
        with pytest.raises(exc):
            solver.solve(**args)
    with pytest.raises(TypeError):
        solver.solve(sm, tr, d)                   # right shapes, not on the GPU


def test_one_shot_solve_checks_data_against_maps_and_trajectory():
    p = mri.AdmmParams(1e-3, 1.0, 2, 2)
    with pytest.raises(ValueError):
        mri.admm_solve(t(NC, NY, NX), t(NK, 2, dtype=F64), t(B, NC + 2, NK), NY, NX, p)
    with pytest.raises(ValueError):
        mri.admm_solve(t(NC, NY, NX), t(NK, 2, dtype=F64), t(B, NC, NK), NY + 1, NX, p)
