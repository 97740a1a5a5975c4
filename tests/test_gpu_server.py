"""Request server (continuous batching) on the GPU, through the C ABI.

* every result equals admm_solve on the same inputs bit for bit, alone and
  inside a mix of other shapes (batch invariance), and matches the oracle
  within the 1e-4 NRMSE bar;
* a budget that holds one request at a time queues the others (no failure);
* a request larger than the pool is refused; cancel works queued and running;
* a request with non-finite data reports MRI_ENUMERIC without touching its
  neighbours' results.
"""
import numpy as np
import pytest
import torch

from oracle import admm as oadmm
from oracle import nudft as onudft
from paper_2006_14080_amd import mri, serve, synth

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _req(nx, ny, nc, spokes, nr, seed, lam=1e-3, beta=1.0, na=4, ncg=3):
    wl = synth.Workload(f"r{seed}", nx, ny, nc, spokes, nr, lam, beta, na, ncg, seed=seed)
    p = synth.make_problem(wl)
    data = (onudft.forward(p.truth[0], p.smaps, p.traj) + p.noise[0]).astype(np.complex64)
    return wl, p, data


def _alone(wl, p, data, prec):
    img, st = mri.admm_solve(_gpu(p.smaps), _gpu(p.traj), _gpu(data[None]), wl.ny, wl.nx,
                             mri.AdmmParams(wl.lam, wl.beta, wl.admm_iters, wl.cg_iters, precision=prec))
    return img.cpu().numpy()[0], st[0]


def _submit(srv, wl, p, data):
    return srv.submit(p.smaps, p.traj, data, mri.AdmmParams(wl.lam, wl.beta, wl.admm_iters, wl.cg_iters))


MIX = [(24, 24, 3, 6, 48, 11), (40, 32, 5, 10, 80, 12), (16, 20, 2, 5, 32, 13), (64, 64, 9, 12, 128, 14)]


@pytest.mark.parametrize("prec", [mri.FP32, mri.BF16X3, mri.FP16X3])
def test_mix_equals_alone_and_oracle(prec):
    reqs = [_req(*m) for m in MIX]
    reqs[1] = _req(40, 32, 5, 10, 80, 12, na=3, ncg=5)      # different counts in the same mix
    with serve.Server(1 << 30, max_slots=8, precision=prec) as srv:
        ids = [_submit(srv, *r) for r in reqs]
        out = srv.run_until_idle(ids)
        info = srv.info()
    assert info["completed"] == len(reqs) and info["pool_used"] == 0
    for rid, (wl, p, data) in zip(ids, reqs):
        img, st = out[rid]
        alone, st1 = _alone(wl, p, data, prec)
        assert np.array_equal(img, alone), wl.name
        assert st["admm_iters"] == wl.admm_iters and st["cg_steps"] == st1["cg_steps"] and st["status"] == 0
        ref = oadmm.admm(data, p.smaps, p.traj, wl.lam, wl.beta, wl.admm_iters, wl.cg_iters).image
        assert np.linalg.norm(img - ref) / np.linalg.norm(ref) <= 1e-4


def test_caller_stream():
    # A server created on the caller's stream runs all its work there and
    # gives the same result as one on a stream of its own.
    a = _req(32, 24, 3, 8, 64, 31, na=3)
    with serve.Server(1 << 28, max_slots=2) as srv:
        ref = srv.run_until_idle([_submit(srv, *a)])
    s = torch.cuda.Stream()
    with serve.Server(1 << 28, max_slots=2, stream=s) as srv:
        out = srv.run_until_idle([_submit(srv, *a)])
    assert np.array_equal(list(ref.values())[0][0], list(out.values())[0][0])


def test_staggered_arrivals_are_batch_invariant():
    # The same request run alone, then admitted while others are mid-solve.
    a = _req(32, 32, 4, 8, 64, 21, na=5)
    others = [_req(48, 40, 3, 9, 96, 22, na=6), _req(20, 28, 6, 7, 56, 23, na=2)]
    with serve.Server(1 << 30, max_slots=4) as srv:
        ra = srv.run_until_idle([_submit(srv, *a)])
    with serve.Server(1 << 30, max_slots=4) as srv:
        i1 = _submit(srv, *others[0])
        srv.step()
        srv.step()
        ia = _submit(srv, *a)
        i2 = _submit(srv, *others[1])
        out = srv.run_until_idle([i1, ia, i2])
        assert srv.info()["graph_captures"] >= 2
    assert np.array_equal(list(ra.values())[0][0], out[ia][0])


def test_small_budget_queues_instead_of_failing():
    reqs = [_req(32, 32, 4, 8, 64, 31 + i, na=2, ncg=2) for i in range(3)]
    one = serve.request_bytes(32, 32, 4, 8 * 64)
    with serve.Server(int(one * 1.5), max_slots=4) as srv:
        ids = [_submit(srv, *r) for r in reqs]
        assert srv.info()["queued"] == 3
        n = srv.step()
        assert n == 1 and srv.info()["queued"] == 2
        out = srv.run_until_idle(ids)
        # a request that can never fit is refused at submit
        big = _req(128, 128, 8, 16, 256, 35, na=1, ncg=1)
        with pytest.raises(mri.MriError) as e:
            _submit(srv, *big)
        assert e.value.code == -2
    for rid, (wl, p, data) in zip(ids, reqs):
        assert np.array_equal(out[rid][0], _alone(wl, p, data, mri.FP32)[0])


def test_cancel_queued_and_running():
    reqs = [_req(24, 24, 2, 6, 48, 41 + i, na=6, ncg=2) for i in range(3)]
    with serve.Server(1 << 28, max_slots=1) as srv:
        ids = [_submit(srv, *r) for r in reqs]
        srv.step()
        assert srv.state(ids[0]) == serve.RUNNING and srv.state(ids[1]) == serve.QUEUED
        srv.cancel(ids[0])
        srv.cancel(ids[1])
        out = srv.run_until_idle([ids[2]])
        info = srv.info()
    assert info["cancelled"] == 2 and info["completed"] == 1 and info["pool_used"] == 0
    wl, p, data = reqs[2]
    assert np.array_equal(out[ids[2]][0], _alone(wl, p, data, mri.FP32)[0])


def test_nonfinite_request_is_isolated():
    good = _req(32, 24, 3, 8, 64, 51)
    bad = _req(32, 24, 3, 8, 64, 52)
    bad_data = bad[2].copy()
    bad_data[1, 17] = np.nan
    with serve.Server(1 << 28, max_slots=4) as srv:
        ig = _submit(srv, *good)
        ib = _submit(srv, bad[0], bad[1], bad_data)
        out = srv.run_until_idle([ig, ib])
    assert out[ib][1]["status"] == -5
    assert out[ig][1]["status"] == 0
    assert np.array_equal(out[ig][0], _alone(*good, mri.FP32)[0])


def test_all_slots_busy_grouped_launches():
    # MRI_SERVER_MAX_SLOTS requests of 16 different shapes in flight at once:
    # every grouped launch carries the maximum of 16 problems; each result
    # still equals its solve alone, bit for bit.
    reqs = [_req(12 + 2 * i, 10 + (3 * i) % 11, 1 + i % 5, 3 + i % 4, 24 + 4 * i, 60 + i, na=2 + i % 3, ncg=2)
            for i in range(16)]
    with serve.Server(1 << 30, max_slots=16) as srv:
        ids = [_submit(srv, *r) for r in reqs]
        srv.step()
        assert srv.info()["active"] == 16
        out = srv.run_until_idle(ids)
    for rid, (wl, p, data) in zip(ids, reqs):
        assert np.array_equal(out[rid][0], _alone(wl, p, data, mri.FP32)[0]), wl.name
