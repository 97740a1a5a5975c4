"""ctypes binding of the request server (mri_server_* in include/mri_admm.h)
and a driver that replays a timed request stream against it.

Argument marshalling only: every reconstruction runs in libmriadmm's kernels.
Inputs are host (numpy) arrays; the server copies them into its own device
pool and hands results back as numpy arrays.
"""
from __future__ import annotations

import ctypes
import time
from typing import Dict, List, Optional

import numpy as np

from . import mri

QUEUED, RUNNING, DONE, UNKNOWN = 0, 1, 2, -1


class MriRequest(ctypes.Structure):
    _fields_ = [("shape", mri.MriShape), ("smaps", ctypes.c_void_p), ("traj", ctypes.c_void_p),
                ("y", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("params", mri.MriAdmmParams)]


class MriServerInfo(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_int32), ("active", ctypes.c_int32), ("completed", ctypes.c_int32),
                ("cancelled", ctypes.c_int32), ("steps", ctypes.c_int64), ("graph_captures", ctypes.c_int64),
                ("pool_bytes", ctypes.c_size_t), ("pool_used", ctypes.c_size_t)]


def _lib():
    lib = mri.load()
    if not getattr(lib, "_server_bound", False):
        vp = ctypes.c_void_p
        lib.mri_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(vp)]
        lib.mri_server_submit.argtypes = [vp, ctypes.POINTER(MriRequest), ctypes.POINTER(ctypes.c_uint64)]
        lib.mri_server_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        lib.mri_server_poll.argtypes = [vp, ctypes.c_uint64, vp, ctypes.POINTER(mri.MriAdmmStats),
                                        ctypes.POINTER(ctypes.c_int)]
        lib.mri_server_cancel.argtypes = [vp, ctypes.c_uint64]
        lib.mri_server_get_info.argtypes = [vp, ctypes.POINTER(MriServerInfo)]
        lib.mri_server_destroy.argtypes = [vp]
        lib.mri_server_request_bytes.argtypes = [ctypes.POINTER(mri.MriShape), ctypes.c_int]
        lib.mri_server_request_bytes.restype = ctypes.c_size_t
        for n in ["mri_server_create", "mri_server_submit", "mri_server_step", "mri_server_poll",
                  "mri_server_cancel", "mri_server_get_info", "mri_server_destroy"]:
            getattr(lib, n).restype = ctypes.c_int
        lib._server_bound = True
    return lib


def request_bytes(nx, ny, nc, nk, precision=mri.FP32) -> int:
    sh = mri.make_shape(nx, ny, nc, nk)
    return int(_lib().mri_server_request_bytes(ctypes.byref(sh), precision))


class Server:
    """One device pool of `budget` bytes and up to `max_slots` concurrent solves.

    `stream`: a torch.cuda.Stream (not the default stream) for all of the
    server's device work, or None for a stream the server owns."""

    def __init__(self, budget: int, max_slots: int = 8, precision: int = mri.FP32, stream=None):
        self.lib = _lib()
        self.precision = precision
        self.h = ctypes.c_void_p()
        self.stream = stream          # kept alive as long as the server
        sp = ctypes.c_void_p(stream.cuda_stream) if stream is not None else ctypes.c_void_p(0)
        mri._check(self.lib.mri_server_create(int(budget), int(max_slots), int(precision), sp,
                                              ctypes.byref(self.h)), "mri_server_create")
        self.shapes: Dict[int, tuple] = {}

    def submit(self, smaps: np.ndarray, traj: np.ndarray, data: np.ndarray, params: mri.AdmmParams,
               x0: Optional[np.ndarray] = None) -> int:
        if smaps.ndim != 3 or traj.ndim != 2 or traj.shape[1] != 2:
            raise ValueError("smaps must be [nc, ny, nx] and traj [nk, 2]")
        nc, ny, nx = smaps.shape
        nk = traj.shape[0]
        if data.size != nc * nk:
            raise ValueError(f"data must hold nc * nk = {nc * nk} samples, got {data.size}")
        if x0 is not None and tuple(x0.shape) != (ny, nx):
            raise ValueError(f"x0 must be [{ny}, {nx}], got {tuple(x0.shape)}")
        smaps = np.ascontiguousarray(smaps, np.complex64)
        traj = np.ascontiguousarray(traj, np.float64)
        data = np.ascontiguousarray(data, np.complex64).reshape(nc, nk)
        req = MriRequest()
        req.shape = mri.make_shape(nx, ny, nc, nk)
        req.smaps = smaps.ctypes.data
        req.traj = traj.ctypes.data
        req.y = data.ctypes.data
        if x0 is not None:
            x0 = np.ascontiguousarray(x0, np.complex64)
            req.x0 = x0.ctypes.data
        else:
            req.x0 = None
        p = params.c()
        p.precision = self.precision
        req.params = p
        rid = ctypes.c_uint64()
        mri._check(self.lib.mri_server_submit(self.h, ctypes.byref(req), ctypes.byref(rid)), "mri_server_submit")
        self.shapes[rid.value] = (ny, nx)
        return rid.value

    def step(self) -> int:
        n = ctypes.c_int()
        mri._check(self.lib.mri_server_step(self.h, ctypes.byref(n)), "mri_server_step")
        return n.value

    def state(self, rid: int) -> int:
        st = ctypes.c_int()
        mri._check(self.lib.mri_server_poll(self.h, rid, None, None, ctypes.byref(st)), "mri_server_poll")
        return st.value

    def collect(self, rid: int):
        """Return (image, stats) if the request is done (releasing it), else None."""
        if self.state(rid) != DONE:
            return None
        ny, nx = self.shapes.pop(rid)
        img = np.empty((ny, nx), np.complex64)
        stats = mri.MriAdmmStats()
        st = ctypes.c_int()
        mri._check(self.lib.mri_server_poll(self.h, rid, img.ctypes.data, ctypes.byref(stats), ctypes.byref(st)),
                   "mri_server_poll")
        return img, dict(admm_iters=stats.admm_iters_run, cg_steps=stats.cg_steps_run, alpha=stats.alpha,
                         tau=stats.tau, status=stats.status)

    def cancel(self, rid: int):
        mri._check(self.lib.mri_server_cancel(self.h, rid), "mri_server_cancel")
        self.shapes.pop(rid, None)

    def info(self) -> dict:
        i = MriServerInfo()
        mri._check(self.lib.mri_server_get_info(self.h, ctypes.byref(i)), "mri_server_get_info")
        return {f: getattr(i, f) for f, _ in MriServerInfo._fields_}

    def close(self):
        if self.h:
            self.lib.mri_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def run_until_idle(self, ids: List[int], max_steps: int = 100000):
        """Step until every id is done; returns {id: (image, stats)}."""
        out = {}
        left = set(ids)
        for _ in range(max_steps):
            if not left:
                break
            self.step()
            for rid in list(left):
                r = self.collect(rid)
                if r is not None:
                    out[rid] = r
                    left.discard(rid)
        if left:
            raise RuntimeError(f"requests {sorted(left)} did not finish")
        return out


def replay(server: Server, arrivals: List[float], payloads: List[dict], progress_s: float = 0.0) -> dict:
    """Feed requests at their arrival times (seconds from start, wall clock)
    while stepping the server; returns latencies and throughput.

    payloads[i] holds the submit() arguments of request i.  With progress_s >
    0 a status line goes to stderr at that interval.
    """
    import sys
    order = np.argsort(arrivals)
    t0 = time.perf_counter()
    last_report = t0
    nxt = 0
    running = {}
    lat = np.zeros(len(arrivals))
    finished = 0
    first_arrival = min(arrivals) if arrivals else 0.0
    while finished < len(arrivals):
        now = time.perf_counter() - t0
        while nxt < len(order) and arrivals[order[nxt]] <= now:
            i = int(order[nxt])
            running[server.submit(**payloads[i])] = i
            nxt += 1
        if not running:
            time.sleep(max(0.0, arrivals[order[nxt]] - now))
            continue
        server.step()
        for rid in list(running):
            r = server.collect(rid)
            if r is not None:
                i = running.pop(rid)
                lat[i] = time.perf_counter() - t0 - arrivals[i]
                finished += 1
        if progress_s > 0 and time.perf_counter() - last_report >= progress_s:
            last_report = time.perf_counter()
            print(f"[replay] t={last_report - t0:.0f}s submitted={nxt} finished={finished}", file=sys.stderr,
                  flush=True)
    wall = time.perf_counter() - t0 - first_arrival
    return {"latency_s": lat, "wall_s": wall, "recons_per_s": len(arrivals) / wall,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "info": server.info()}
