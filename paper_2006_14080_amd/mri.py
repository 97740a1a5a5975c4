"""ctypes binding of libmriadmm (C ABI in include/mri_admm.h).

Argument marshalling only: tensors must already live on the GPU; every step
of the computation runs in the library's HIP kernels on the current torch
stream.  The library is loaded on first use and a missing build raises --
there is no CPU fallback.

Shapes (complex64 unless noted):
  image  [B, ny, nx]          smaps [nc, ny, nx] or [B, nc, ny, nx]
  traj   [nk, 2] or [B, nk, 2] float64, radians per pixel, column 0 <-> x
  data   [B, nc, nk]          grad  [B, 2, ny, nx]
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmriadmm.so")

FP32 = 0
BF16X3 = 1
FP16X3 = 2
NUFFT = 3            # admm_solve only: F by the NUFFT operator (width 6, oversampling 2, FP32)
PRECISIONS = {"fp32": FP32, "bf16x3": BF16X3, "fp16x3": FP16X3, "nufft": NUFFT}
PRECISION_NAMES = {v: k for k, v in PRECISIONS.items()}

OP_FORWARD, OP_ADJOINT, OP_ADMM = 0, 1, 2

ERRORS = {0: "MRI_OK", -1: "MRI_EINVAL", -2: "MRI_ENOMEM", -3: "MRI_EHIP",
          -4: "MRI_ENOTSUP", -5: "MRI_ENUMERIC"}


class MriShape(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("ncoils", ctypes.c_int32),
                ("nk", ctypes.c_int64), ("batch", ctypes.c_int32),
                ("traj_batched", ctypes.c_int32), ("smaps_batched", ctypes.c_int32)]


class MriAdmmParams(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_double), ("beta", ctypes.c_double),
                ("admm_iters", ctypes.c_int32), ("cg_iters", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("precision", ctypes.c_int32), ("cg_warm_start", ctypes.c_int32)]


class MriAdmmStats(ctypes.Structure):
    _fields_ = [("admm_iters_run", ctypes.c_int32), ("cg_steps_run", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("tau", ctypes.c_double),
                ("status", ctypes.c_int32), ("pad", ctypes.c_int32)]


class MriNufftParams(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("pad", ctypes.c_int32), ("sigma", ctypes.c_double)]


STATS_BYTES = ctypes.sizeof(MriAdmmStats)

EXPORTS = ["nudft_forward", "nudft_forward_noalloc", "mri_noalloc_scratch_bytes", "nudft_adjoint", "nudft_adjoint_prepare", "nudft_adjoint_prepared",
           "tv_forward", "tv_adjoint", "admm_solve", "mri_workspace_bytes", "mri_adjoint_split",
           "mri_strerror", "mri_last_hip_error", "mri_nufft_workspace_bytes", "nufft_prepare", "nufft_forward",
           "nufft_adjoint"]

_lib = None


class MriError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)}{(' - ' + detail) if detail else ''}")


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2006_14080_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
    shp = ctypes.POINTER(MriShape)
    prm = ctypes.POINTER(MriAdmmParams)
    lib.nudft_forward.argtypes = [shp, vp, vp, vp, vp, i32, vp, sz, vp]
    lib.nudft_adjoint.argtypes = [shp, vp, vp, vp, vp, i32, vp, sz, vp]
    lib.nudft_forward_noalloc.argtypes = [shp, vp, vp, vp, vp, i32, vp]
    lib.nudft_forward_noalloc.restype = i32
    lib.mri_noalloc_scratch_bytes.argtypes = []
    lib.mri_noalloc_scratch_bytes.restype = sz
    lib.nudft_adjoint_prepare.argtypes = [shp, vp, vp, sz, vp]
    lib.nudft_adjoint_prepared.argtypes = [shp, vp, vp, vp, vp, i32, vp, sz, vp]
    lib.tv_forward.argtypes = [shp, vp, vp, vp]
    lib.tv_adjoint.argtypes = [shp, vp, vp, vp]
    lib.admm_solve.argtypes = [shp, vp, vp, vp, vp, prm, vp, vp, vp, sz, vp]
    lib.mri_workspace_bytes.argtypes = [shp, i32, prm]
    lib.mri_workspace_bytes.restype = sz
    nup = ctypes.POINTER(MriNufftParams)
    lib.mri_nufft_workspace_bytes.argtypes = [shp, nup]
    lib.mri_nufft_workspace_bytes.restype = sz
    lib.nufft_prepare.argtypes = [shp, vp, nup, vp, sz, vp]
    lib.nufft_forward.argtypes = [shp, vp, vp, vp, nup, vp, sz, vp]
    lib.nufft_adjoint.argtypes = [shp, vp, vp, vp, nup, vp, sz, vp]
    for name in ["nufft_prepare", "nufft_forward", "nufft_adjoint"]:
        getattr(lib, name).restype = i32
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.mri_adjoint_split.argtypes = [shp, i32p, i32p, i32p]
    lib.mri_adjoint_split.restype = i32
    lib.mri_strerror.argtypes = [i32]
    lib.mri_strerror.restype = ctypes.c_char_p
    lib.mri_last_hip_error.argtypes = []
    lib.mri_last_hip_error.restype = ctypes.c_char_p
    for name in ["nudft_forward", "nudft_adjoint", "nudft_adjoint_prepare", "nudft_adjoint_prepared",
                 "tv_forward", "tv_adjoint", "admm_solve"]:
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != 0:
        detail = ""
        if rc == -3:
            detail = load().mri_last_hip_error().decode()
        raise MriError(rc, where, detail)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _need(t: torch.Tensor, dtype, name: str, shape=None):
    """Check one tensor argument before any library call: type, dtype, exact
    shape (when given) and contiguity.  A tensor that does not match the shape
    the library is told about would make its kernels read or write outside
    it, so every mismatch raises here and nothing is launched."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(int(v) for v in shape):
        raise ValueError(f"{name} must have shape {tuple(int(v) for v in shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _on_gpu(device=None, **tensors):
    """Every tensor (None skipped) is a GPU tensor on one device (`device`
    when given, else the first tensor's).  Called after the shape checks."""
    for name, t in tensors.items():
        if t is None:
            continue
        if not t.is_cuda:
            raise TypeError(f"{name} must be a GPU tensor")
        if device is None:
            device = t.device
        elif t.device != torch.device(device):
            raise ValueError(f"{name} is on {t.device}, expected {device}")


def _check_inputs(sh: "MriShape", smaps: torch.Tensor, traj: torch.Tensor):
    """smaps and traj against a shape: [nc, ny, nx] or [B, nc, ny, nx], and
    [nk, 2] or [B, nk, 2] as its *_batched flags say."""
    sm = (sh.ncoils, sh.ny, sh.nx)
    tr = (sh.nk, 2)
    _need(smaps, torch.complex64, "smaps", ((sh.batch,) + sm) if sh.smaps_batched else sm)
    _need(traj, torch.float64, "traj", ((sh.batch,) + tr) if sh.traj_batched else tr)


def make_shape(nx, ny, nc, nk, batch=1, traj_batched=False, smaps_batched=False) -> MriShape:
    return MriShape(int(nx), int(ny), int(nc), int(nk), int(batch), int(traj_batched), int(smaps_batched))


def shape_of(image_shape, smaps: torch.Tensor, traj: torch.Tensor) -> MriShape:
    """The MriShape of a [B, ny, nx] image with these coil maps and trajectory
    (batched when they carry a leading slice axis)."""
    if len(image_shape) != 3:
        raise ValueError(f"image must be [B, ny, nx], got {tuple(image_shape)}")
    b, ny, nx = (int(v) for v in image_shape)
    if not isinstance(smaps, torch.Tensor) or not isinstance(traj, torch.Tensor):
        raise TypeError("smaps and traj must be torch.Tensors")
    if smaps.dim() not in (3, 4) or traj.dim() not in (2, 3):
        raise ValueError("smaps must be [nc, ny, nx] or [B, nc, ny, nx]; traj [nk, 2] or [B, nk, 2]")
    smaps_batched = smaps.dim() == 4
    traj_batched = traj.dim() == 3
    nc = smaps.shape[-3]
    nk = traj.shape[-2]
    if tuple(smaps.shape[-2:]) != (ny, nx):
        raise ValueError("smaps do not match the image grid")
    if smaps_batched and smaps.shape[0] != b:
        raise ValueError("batched smaps must have one map set per slice")
    if traj_batched and traj.shape[0] != b:
        raise ValueError("batched traj must have one trajectory per slice")
    if traj.shape[-1] != 2:
        raise ValueError("traj must be [..., nk, 2]")
    return make_shape(nx, ny, nc, nk, b, traj_batched, smaps_batched)


def workspace_bytes(shape: MriShape, op: int, params: Optional[MriAdmmParams] = None) -> int:
    lib = load()
    return int(lib.mri_workspace_bytes(ctypes.byref(shape), op,
                                       ctypes.byref(params) if params is not None else None))


def adjoint_split(shape: MriShape) -> dict:
    """The adjoint's sample-range split for a shape: {'ksplit', 'kper',
    'planes'} (partial images per slice)."""
    ks, kp, pl = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().mri_adjoint_split(ctypes.byref(shape), ctypes.byref(ks), ctypes.byref(kp), ctypes.byref(pl)),
           "mri_adjoint_split")
    return {"ksplit": ks.value, "kper": kp.value, "planes": pl.value}


def _workspace(shape, op, params=None, device=None):
    n = workspace_bytes(shape, op, params)
    if n == 0:
        return None, 0
    return torch.empty(n, dtype=torch.uint8, device=device), n


def nudft_forward(image: torch.Tensor, smaps: torch.Tensor, traj: torch.Tensor,
                  precision: int = FP32, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = F(image), eq. (1): [B, ny, nx] -> [B, nc, nk]."""
    lib = load()
    _need(image, torch.complex64, "image")
    sh = shape_of(image.shape, smaps, traj)
    _check_inputs(sh, smaps, traj)
    if out is not None:
        _need(out, torch.complex64, "out", (sh.batch, sh.ncoils, sh.nk))
    _on_gpu(image=image, smaps=smaps, traj=traj, out=out)
    if out is None:
        out = torch.empty((sh.batch, sh.ncoils, sh.nk), dtype=torch.complex64, device=image.device)
    ws, n = _workspace(sh, OP_FORWARD, device=image.device)
    _check(lib.nudft_forward(ctypes.byref(sh), _ptr(image), _ptr(smaps), _ptr(traj), _ptr(out),
                             precision, _ptr(ws), n, _stream()), "nudft_forward")
    return out


def nudft_forward_noalloc(image: torch.Tensor, smaps: torch.Tensor, traj: torch.Tensor,
                          precision: int = FP32, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """nudft_forward without a workspace: the library's static device scratch
    (mri_noalloc_scratch_bytes) holds the coil-weighted images.  Calls that
    overlap on one GPU race for that scratch."""
    lib = load()
    _need(image, torch.complex64, "image")
    sh = shape_of(image.shape, smaps, traj)
    _check_inputs(sh, smaps, traj)
    if out is not None:
        _need(out, torch.complex64, "out", (sh.batch, sh.ncoils, sh.nk))
    _on_gpu(image=image, smaps=smaps, traj=traj, out=out)
    if out is None:
        out = torch.empty((sh.batch, sh.ncoils, sh.nk), dtype=torch.complex64, device=image.device)
    _check(lib.nudft_forward_noalloc(ctypes.byref(sh), _ptr(image), _ptr(smaps), _ptr(traj), _ptr(out),
                                     precision, _stream()), "nudft_forward_noalloc")
    return out


def nudft_adjoint(data: torch.Tensor, smaps: torch.Tensor, traj: torch.Tensor, ny: int, nx: int,
                  precision: int = FP32, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = F^H(data): [B, nc, nk] -> [B, ny, nx]."""
    lib = load()
    if not isinstance(data, torch.Tensor) or data.dim() != 3:
        raise ValueError("data must be a [B, nc, nk] tensor")
    b = data.shape[0]
    sh = shape_of((b, ny, nx), smaps, traj)
    _need(data, torch.complex64, "data", (b, sh.ncoils, sh.nk))
    _check_inputs(sh, smaps, traj)
    if out is not None:
        _need(out, torch.complex64, "out", (b, ny, nx))
    _on_gpu(data=data, smaps=smaps, traj=traj, out=out)
    if out is None:
        out = torch.empty((b, ny, nx), dtype=torch.complex64, device=data.device)
    ws, n = _workspace(sh, OP_ADJOINT, device=data.device)
    _check(lib.nudft_adjoint(ctypes.byref(sh), _ptr(data), _ptr(smaps), _ptr(traj), _ptr(out),
                             precision, _ptr(ws), n, _stream()), "nudft_adjoint")
    return out


class AdjointPlan:
    """F^H for a fixed trajectory: the phase tables are built once
    (nudft_adjoint_prepare) into a workspace this object owns, and every call
    applies nudft_adjoint_prepared (bit-identical to nudft_adjoint)."""

    def __init__(self, smaps: torch.Tensor, traj: torch.Tensor, ny: int, nx: int, batch: int = 1,
                 precision: int = FP32):
        self.smaps, self.traj, self.precision = smaps, traj, precision
        self.shape = shape_of((batch, ny, nx), smaps, traj)
        _check_inputs(self.shape, smaps, traj)
        _on_gpu(smaps=smaps, traj=traj)
        self.ws, self.ws_bytes = _workspace(self.shape, OP_ADJOINT, device=smaps.device)
        _check(load().nudft_adjoint_prepare(ctypes.byref(self.shape), _ptr(traj), _ptr(self.ws),
                                            self.ws_bytes, _stream()), "nudft_adjoint_prepare")

    def __call__(self, data: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        sh = self.shape
        _need(data, torch.complex64, "data", (sh.batch, sh.ncoils, sh.nk))
        if out is not None:
            _need(out, torch.complex64, "out", (sh.batch, sh.ny, sh.nx))
        _on_gpu(self.smaps.device, data=data, out=out)
        if out is None:
            out = torch.empty((sh.batch, sh.ny, sh.nx), dtype=torch.complex64, device=data.device)
        _check(load().nudft_adjoint_prepared(ctypes.byref(sh), _ptr(data), _ptr(self.smaps), _ptr(self.traj),
                                             _ptr(out), self.precision, _ptr(self.ws), self.ws_bytes,
                                             _stream()), "nudft_adjoint_prepared")
        return out


class NufftPlan:
    """The NUFFT operator (nufft_prepare / nufft_forward / nufft_adjoint) for
    fixed maps, trajectory, image size and batch: the plan and the grid live in
    a workspace this object owns, built once here."""

    def __init__(self, smaps: torch.Tensor, traj: torch.Tensor, ny: int, nx: int, batch: int = 1,
                 width: int = 6, sigma: float = 2.0):
        self.shape = shape_of((batch, ny, nx), smaps, traj)
        _check_inputs(self.shape, smaps, traj)
        _on_gpu(smaps=smaps, traj=traj)
        self.smaps, self.traj = smaps, traj
        self.params = MriNufftParams(int(width), 0, float(sigma))
        lib = load()
        n = int(lib.mri_nufft_workspace_bytes(ctypes.byref(self.shape), ctypes.byref(self.params)))
        if n == 0:
            raise ValueError("unsupported NUFFT shape or parameters")
        self.ws = torch.empty(n, dtype=torch.uint8, device=smaps.device)
        self.ws_bytes = n
        _check(lib.nufft_prepare(ctypes.byref(self.shape), _ptr(traj), ctypes.byref(self.params), _ptr(self.ws),
                                 n, _stream()), "nufft_prepare")

    def forward(self, image: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y ~ F(image): [B, ny, nx] -> [B, nc, nk]."""
        sh = self.shape
        _need(image, torch.complex64, "image", (sh.batch, sh.ny, sh.nx))
        if out is not None:
            _need(out, torch.complex64, "out", (sh.batch, sh.ncoils, sh.nk))
        _on_gpu(self.smaps.device, image=image, out=out)
        if out is None:
            out = torch.empty((sh.batch, sh.ncoils, sh.nk), dtype=torch.complex64, device=image.device)
        _check(load().nufft_forward(ctypes.byref(sh), _ptr(image), _ptr(self.smaps), _ptr(out),
                                    ctypes.byref(self.params), _ptr(self.ws), self.ws_bytes, _stream()),
               "nufft_forward")
        return out

    def adjoint(self, data: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """x ~ F^H(data): [B, nc, nk] -> [B, ny, nx]."""
        sh = self.shape
        _need(data, torch.complex64, "data", (sh.batch, sh.ncoils, sh.nk))
        if out is not None:
            _need(out, torch.complex64, "out", (sh.batch, sh.ny, sh.nx))
        _on_gpu(self.smaps.device, data=data, out=out)
        if out is None:
            out = torch.empty((sh.batch, sh.ny, sh.nx), dtype=torch.complex64, device=data.device)
        _check(load().nufft_adjoint(ctypes.byref(sh), _ptr(data), _ptr(self.smaps), _ptr(out),
                                    ctypes.byref(self.params), _ptr(self.ws), self.ws_bytes, _stream()),
               "nufft_adjoint")
        return out


def tv_forward(image: torch.Tensor) -> torch.Tensor:
    """g = Theta(image): [B, ny, nx] -> [B, 2, ny, nx]."""
    lib = load()
    _need(image, torch.complex64, "image")
    if image.dim() != 3:
        raise ValueError(f"image must be [B, ny, nx], got {tuple(image.shape)}")
    _on_gpu(image=image)
    b, ny, nx = image.shape
    sh = make_shape(nx, ny, 1, 1, b)
    g = torch.empty((b, 2, ny, nx), dtype=torch.complex64, device=image.device)
    _check(lib.tv_forward(ctypes.byref(sh), _ptr(image), _ptr(g), _stream()), "tv_forward")
    return g


def tv_adjoint(grad: torch.Tensor) -> torch.Tensor:
    """x = Theta^H(grad): [B, 2, ny, nx] -> [B, ny, nx]."""
    lib = load()
    _need(grad, torch.complex64, "grad")
    if grad.dim() != 4 or grad.shape[1] != 2:
        raise ValueError(f"grad must be [B, 2, ny, nx], got {tuple(grad.shape)}")
    _on_gpu(grad=grad)
    b, two, ny, nx = grad.shape
    sh = make_shape(nx, ny, 1, 1, b)
    x = torch.empty((b, ny, nx), dtype=torch.complex64, device=grad.device)
    _check(lib.tv_adjoint(ctypes.byref(sh), _ptr(grad), _ptr(x), _stream()), "tv_adjoint")
    return x


@dataclasses.dataclass
class AdmmParams:
    lam: float
    beta: float
    admm_iters: int
    cg_iters: int
    rtol: float = 0.0
    atol: float = 0.0
    precision: int = FP32
    cg_warm_start: bool = True

    def c(self) -> MriAdmmParams:
        return MriAdmmParams(float(self.lam), float(self.beta), int(self.admm_iters), int(self.cg_iters),
                             float(self.rtol), float(self.atol), int(self.precision), int(self.cg_warm_start))


class AdmmSolver:
    """Reusable admm_solve launcher: owns its workspace, so repeated solves of
    one shape allocate nothing after construction."""

    def __init__(self, shape: MriShape, params: AdmmParams, device="cuda"):
        self.shape = shape
        self.params = params
        self._cp = params.c()
        n = workspace_bytes(shape, OP_ADMM, self._cp)
        self.ws = torch.empty(max(n, 1), dtype=torch.uint8, device=device)
        self.ws_bytes = n
        self.stats_buf = torch.zeros(shape.batch * STATS_BYTES, dtype=torch.uint8, device=device)

    def solve(self, smaps, traj, data, x0=None, out=None) -> torch.Tensor:
        lib = load()
        sh = self.shape
        dev = self.ws.device
        img = (sh.batch, sh.ny, sh.nx)
        _check_inputs(sh, smaps, traj)
        _need(data, torch.complex64, "data", (sh.batch, sh.ncoils, sh.nk))
        if x0 is not None:
            _need(x0, torch.complex64, "x0", img)
        if out is not None:
            _need(out, torch.complex64, "out", img)
        _on_gpu(dev, smaps=smaps, traj=traj, data=data, x0=x0, out=out)
        if out is None:
            out = torch.empty(img, dtype=torch.complex64, device=dev)
        _check(lib.admm_solve(ctypes.byref(sh), _ptr(smaps), _ptr(traj), _ptr(data), _ptr(x0),
                              ctypes.byref(self._cp), _ptr(out), _ptr(self.stats_buf),
                              _ptr(self.ws), self.ws_bytes, _stream()), "admm_solve")
        return out

    def stats(self):
        """Per-slice solve report (synchronises the stream)."""
        raw = self.stats_buf.cpu().numpy().tobytes()
        out = []
        for b in range(self.shape.batch):
            s = MriAdmmStats.from_buffer_copy(raw[b * STATS_BYTES:(b + 1) * STATS_BYTES])
            out.append(dict(admm_iters=s.admm_iters_run, cg_steps=s.cg_steps_run, alpha=s.alpha,
                            tau=s.tau, status=s.status))
        return out


def admm_solve(smaps, traj, data, ny, nx, params: AdmmParams, x0=None):
    """One-shot ADMM-TV reconstruction (Alg. 4).  Returns (image, stats)."""
    if not isinstance(data, torch.Tensor) or data.dim() != 3:
        raise ValueError("data must be a [B, nc, nk] tensor")
    sh = shape_of((data.shape[0], ny, nx), smaps, traj)
    _check_inputs(sh, smaps, traj)
    solver = AdmmSolver(sh, params, device=data.device)
    img = solver.solve(smaps, traj, data, x0)
    return img, solver.stats()
