"""Seeded synthetic inputs for ADMM-TV reconstruction of radial multi-coil MRI.

This module only draws inputs: an ellipse phantom (the image rho of eq. (1)),
Gaussian coil sensitivities s, a golden-angle radial trajectory k, complex
Gaussian noise, and the parameter sets of the workloads.  It holds none of the
reconstruction arithmetic (no DFT, no finite differences, no solver), so both
the FP64 test oracle and the GPU path can take their inputs from it.

Stand-ins: the paper reconstructs scanner phantom data acquired with a
12-channel coil along radial readouts (Sec. V, Sec. VI).  Those data are not
available, so these generators produce inputs with the same structure:
a piecewise-constant phantom, smooth multi-coil sensitivities and an
undersampled radial trajectory.

Conventions (shared by every consumer):
  * image   [ny][nx] complex64, x (column) fastest; pixel (i, j) sits at the
    centred integer offsets y = i - ny//2, x = j - nx//2;
  * smaps   [nc][ny][nx] complex64;
  * traj    [nk][2] float64 in radians per pixel, column 0 pairs with x and
    column 1 with y; sample index = spoke * n_readout + readout;
  * data    [nc][nk] complex64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

GOLDEN_ANGLE = math.pi * (math.sqrt(5.0) - 1.0) / 2.0  # 111.246 degrees, in rad


def _centred(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) - (n // 2)


def ellipse_phantom(nx: int, ny: int, seed: int, n_ellipses: int = 10) -> np.ndarray:
    """Additive random-ellipse phantom, real values stored as complex64.

    Normalised coordinates u = x / (nx/2), v = y / (ny/2).  Each ellipse has
    centre ~ U(-0.45, 0.45)^2, semi-axes ~ U(0.08, 0.45), rotation ~ U(0, pi)
    and amplitude ~ U(0.2, 1.0); a pixel belongs to it when its rotated,
    axis-scaled offset has norm <= 1.
    """
    rng = np.random.default_rng(seed)
    u = _centred(nx)[None, :] / (nx / 2.0)
    v = _centred(ny)[:, None] / (ny / 2.0)
    img = np.zeros((ny, nx), dtype=np.float64)
    for _ in range(n_ellipses):
        cx, cy = rng.uniform(-0.45, 0.45, size=2)
        a, b = rng.uniform(0.08, 0.45, size=2)
        th = rng.uniform(0.0, math.pi)
        amp = rng.uniform(0.2, 1.0)
        du, dv = u - cx, v - cy
        c, s = math.cos(th), math.sin(th)
        p = (c * du + s * dv) / a
        q = (-s * du + c * dv) / b
        img += amp * ((p * p + q * q) <= 1.0)
    return img.astype(np.complex64)


def coil_maps(nx: int, ny: int, nc: int) -> np.ndarray:
    """Gaussian coil sensitivities centred on the edge circle, complex64.

    Coil g sits at angle phi = 2*pi*g/nc, centre (nx/2 cos phi, ny/2 sin phi)
    in pixel units, width sigma = (nx/3, ny/3), and carries the phase
    exp(i*phi).  The maps are not normalised.
    """
    x = _centred(nx)[None, :]
    y = _centred(ny)[:, None]
    sx, sy = nx / 3.0, ny / 3.0
    out = np.empty((nc, ny, nx), dtype=np.complex128)
    for g in range(nc):
        phi = 2.0 * math.pi * g / nc
        cx, cy = (nx / 2.0) * math.cos(phi), (ny / 2.0) * math.sin(phi)
        mag = np.exp(-((x - cx) ** 2 / (2 * sx * sx) + (y - cy) ** 2 / (2 * sy * sy)))
        out[g] = mag * complex(math.cos(phi), math.sin(phi))
    return out.astype(np.complex64)


def radial_trajectory(n_spokes: int, n_readout: int) -> np.ndarray:
    """Golden-angle radial trajectory in radians per pixel, float64 [nk][2].

    Spoke s has angle s * GOLDEN_ANGLE; readout j sits at radius
    -pi + 2*pi*j/n_readout, so radii cover [-pi, pi).
    """
    th = np.arange(n_spokes, dtype=np.float64) * GOLDEN_ANGLE
    r = -math.pi + 2.0 * math.pi * np.arange(n_readout, dtype=np.float64) / n_readout
    kx = r[None, :] * np.cos(th)[:, None]
    ky = r[None, :] * np.sin(th)[:, None]
    return np.ascontiguousarray(np.stack([kx.ravel(), ky.ravel()], axis=1))


def cartesian_trajectory(nx: int, ny: int) -> np.ndarray:
    """Every point of the nx-by-ny Cartesian grid, float64 [ny*nx][2].

    Sample index = iy * nx + ix with omega = 2*pi*(i - n//2)/n per axis.
    """
    wx = 2.0 * math.pi * _centred(nx) / nx
    wy = 2.0 * math.pi * _centred(ny) / ny
    gx, gy = np.meshgrid(wx, wy)
    return np.ascontiguousarray(np.stack([gx.ravel(), gy.ravel()], axis=1))


def complex_noise(shape, sigma: float, seed: int) -> np.ndarray:
    """sigma * (n1 + i n2) with n1, n2 ~ N(0, 1), complex128."""
    rng = np.random.default_rng(seed)
    return sigma * (rng.standard_normal(shape) + 1j * rng.standard_normal(shape))


def random_complex(shape, seed: int, dtype=np.complex64) -> np.ndarray:
    """Standard complex Gaussian test vector (re, im ~ N(0, 1))."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


def random_trajectory(nk: int, seed: int) -> np.ndarray:
    """Uniform random k-space points in [-pi, pi)^2, float64 [nk][2]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-math.pi, math.pi, size=(nk, 2))


@dataclasses.dataclass(frozen=True)
class Workload:
    """One reconstruction problem shape plus its ADMM parameters.

    ``beta`` is the augmented-Lagrangian penalty of eq. (5); the threshold of
    eq. (9) is lam / beta.
    """
    name: str
    nx: int
    ny: int
    nc: int
    n_spokes: int
    n_readout: int
    lam: float
    beta: float
    admm_iters: int
    cg_iters: int
    batch: int = 1
    seed: int = 0
    sigma: float = 1e-3
    rtol: float = 0.0
    atol: float = 0.0

    @property
    def nk(self) -> int:
        return self.n_spokes * self.n_readout

    @property
    def nudft_calls(self) -> int:
        """NUDFT applications per solve: one F^H d plus two per A-application."""
        return 1 + 2 * self.admm_iters * (1 + self.cg_iters)

    @property
    def nudft_flop(self) -> float:
        """Algorithmic flop of one NUDFT call: 8 per complex multiply-add."""
        return 8.0 * self.nk * self.nx * self.ny * self.nc * self.batch


# The workloads: 32x32 / 256x256 single slices, a 32-slice 384x384 batch.
ADMM32 = Workload("admm_tv_32x32_c4_r16x64_10x3", 32, 32, 4, 16, 64,
                  1e-3, 1.0, 10, 3, seed=101)
ADMM256 = Workload("admm_tv_256x256_c8_r64x512_30x5", 256, 256, 8, 64, 512,
                   1e-3, 1.0, 30, 5, seed=202)
SLICES384 = Workload("admm_tv_32x384x384_c16_r128x768_40x5", 384, 384, 16, 128, 768,
                     5e-4, 1.0, 40, 5, batch=32, seed=400)

# Paper-shaped stand-ins (Sec. V): a 128 x 64 grid with a 12-channel coil.
# Fully sampled radial data (101 spokes x 128 samples) for the "inverse DFT"
# accuracy experiment, and the x8-undersampled set (13 spokes x 128 samples)
# reconstructed with the Table I parameters (lambda 1e-7, beta 1, relative
# tolerance 1e-4 over at most 5 ADMM iterations, CG absolute tolerance 1e-6
# over at most 20 steps).
INVDFT128x64 = Workload("inverse_dft_128x64_c12_r101x128", 128, 64, 12, 101, 128,
                        0.0, 1.0, 0, 0, seed=606)
TABLE1_128x64 = Workload("admm_tv_table1_128x64_c12_r13x128", 128, 64, 12, 13, 128,
                         1e-7, 1.0, 5, 20, seed=707, rtol=1e-4, atol=1e-6)
# The large-image scaling case of Sec. VI: a 1024 x 512 grid, 12 coils,
# 103,424 samples per coil (101 spokes x 1024 samples after x8
# undersampling), Table I parameters.
TABLE1_1024x512 = Workload("admm_tv_table1_1024x512_c12_r101x1024", 1024, 512, 12, 101, 1024,
                           1e-7, 1.0, 5, 20, seed=808, rtol=1e-4, atol=1e-6)


def kspace_shards(nk: int, parts: int) -> List[Tuple[int, int]]:
    """Contiguous sample ranges [lo, hi) splitting nk samples into `parts`
    near-equal pieces (the k-space decomposition of Sec. IV-A, where each
    core holds one range of every coil's samples)."""
    bounds = [nk * p // parts for p in range(parts + 1)]
    return list(zip(bounds[:-1], bounds[1:]))


@dataclasses.dataclass
class Problem:
    """Inputs of one (possibly batched) reconstruction, as numpy arrays.

    ``truth`` [B][ny][nx], ``smaps`` [nc][ny][nx] (shared across the batch),
    ``traj`` [nk][2] (shared), ``noise`` [B][nc][nk] (complex128; the data are
    F(truth) + noise, formed by whichever side consumes them).
    """
    wl: Workload
    truth: np.ndarray
    smaps: np.ndarray
    traj: np.ndarray
    noise: np.ndarray


def make_problem(wl: Workload, batch: Optional[int] = None) -> Problem:
    """Draw the phantom(s), maps, trajectory and noise for a workload.

    Slice b of a batch uses phantom seed wl.seed + b; its noise seed is that
    phantom seed + 1 offset by 1000 so no two draws share a stream.
    """
    nb = wl.batch if batch is None else batch
    truth = np.stack([slice_phantom(wl, b) for b in range(nb)])
    smaps = coil_maps(wl.nx, wl.ny, wl.nc)
    traj = radial_trajectory(wl.n_spokes, wl.n_readout)
    noise = np.stack([slice_noise(wl, b) for b in range(nb)])
    return Problem(wl, truth, smaps, traj, noise)


def slice_phantom(wl: Workload, b: int) -> np.ndarray:
    """Phantom of slice b of a workload (as in make_problem), [ny][nx]."""
    return ellipse_phantom(wl.nx, wl.ny, wl.seed + b)


def slice_noise(wl: Workload, b: int) -> np.ndarray:
    """Noise of slice b of a workload (as in make_problem), complex128 [nc][nk]."""
    return complex_noise((wl.nc, wl.nk), wl.sigma, 1000 + wl.seed + b + 1)


@dataclasses.dataclass(frozen=True)
class Request:
    """One request of a served stream: arrival time (s) and its workload."""
    rid: int
    arrival: float
    wl: Workload


def request_stream(n_requests: int = 200, rate: float = 20.0, seed: int = 5,
                   admm_iters: int = 30, cg_iters: int = 5,
                   sizes=(128, 256, 384), coils=(4, 32), spokes=(32, 128),
                   lam: float = 1e-3, beta: float = 1.0) -> List[Request]:
    """Poisson arrivals of mixed-shape requests.

    Image side N ~ U{sizes}, coils ~ U{coils[0]..coils[1]}, spokes ~
    U{spokes[0]..spokes[1]}, readout = 2N (2x oversampled); request r uses
    phantom seed 5000 + r.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate)
        n = int(rng.choice(sizes))
        nc = int(rng.integers(coils[0], coils[1] + 1))
        ns = int(rng.integers(spokes[0], spokes[1] + 1))
        wl = Workload(f"req{r}_{n}x{n}_c{nc}_r{ns}x{2 * n}", n, n, nc, ns, 2 * n,
                      lam, beta, admm_iters, cg_iters, seed=5000 + r)
        out.append(Request(r, t, wl))
    return out
