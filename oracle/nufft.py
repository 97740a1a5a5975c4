"""Non-uniform FFT approximation of the multi-coil NUDFT, FP64 (test oracle only).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper's CPU and GPU comparison systems apply the forward model with a
NUFFT (gridding and an FFT, Sec. VII and Table II), the O(N log N)
alternative to the dense DFT that the paper names as the way to larger
images.  This module computes it plainly: with a Kaiser-Bessel interpolation
kernel of width W grid points on a grid oversampled by sigma,

  forward  d(w) ~ sum_m psi(t - m) U[m],   U = FFT_G( s (.) rho / Psi ),
  adjoint  rho ~ sum_g conj(s_g) (.) crop( IFFT_G( sum_k d_k psi(t_k - m) ) ) / Psi,

per axis t = w G / (2 pi) (the sample's position in grid units), m the
integer grid points within W/2 of t (taken modulo G), G the grid size, Psi
the kernel's continuous Fourier transform at the pixel offsets (the
deapodisation), FFT_G the unnormalised G-point DFT with exp(-i 2 pi m x / G)
and IFFT_G its conjugate transpose.  The kernel and its transform:

  psi(u) = I0(beta sqrt(1 - (2u/W)^2))  for |u| <= W/2, else 0,
  Psi(f) = W sinh(sqrt(beta^2 - (pi W f)^2)) / sqrt(beta^2 - (pi W f)^2),

with beta = pi sqrt(W^2 (sigma - 1/2)^2 / sigma^2 - 0.8) (Beatty, Nishimura
and Pauly, IEEE TMI 2005).  The grid is the smallest power of two at least
sigma times the image side.  Since the FFT's exp(-i 2 pi m x / G) with the
kernel's shift reproduces exp(-i w x) up to the kernel's aliasing, the
forward approximates eq. (1) and the adjoint is its exact adjoint.
Image offsets are centred (x = j - n//2) as in oracle.nudft.
"""
import math

import numpy as np


def grid_size(n, sigma):
    """Smallest power of two >= sigma * n."""
    g = 1
    while g < sigma * n:
        g *= 2
    return g


def kb_beta(width, sigma):
    return math.pi * math.sqrt(width * width * (sigma - 0.5) ** 2 / (sigma * sigma) - 0.8)


def kb_kernel(u, width, beta):
    """psi(u) for an array u of offsets in grid units (0 outside |u| <= W/2)."""
    u = np.asarray(u, dtype=np.float64)
    z = 1.0 - (2.0 * u / width) ** 2
    out = np.zeros_like(u)
    inside = z >= 0.0
    out[inside] = np.i0(beta * np.sqrt(z[inside]))
    return out


def kb_transform(f, width, beta):
    """Psi(f), the Fourier transform int psi(u) exp(i 2 pi u f) du (real, even)."""
    f = np.asarray(f, dtype=np.float64)
    a = beta * beta - (math.pi * width * f) ** 2
    out = np.empty_like(f)
    pos = a > 0
    r = np.sqrt(a[pos])
    out[pos] = width * np.sinh(r) / r
    neg = ~pos
    r = np.sqrt(-a[neg])
    out[neg] = width * np.where(r > 0, np.sin(r) / np.where(r > 0, r, 1.0), 1.0)
    return out


class Plan:
    """Grid sizes, kernel and deapodisation for an ny x nx image and a trajectory."""

    def __init__(self, nx, ny, traj, width=6, sigma=2.0):
        self.nx, self.ny = nx, ny
        self.width = int(width)
        self.sigma = float(sigma)
        self.gx, self.gy = grid_size(nx, sigma), grid_size(ny, sigma)
        # the kernel is designed for the oversampling actually used on each axis
        self.bx = kb_beta(self.width, self.gx / nx)
        self.by = kb_beta(self.width, self.gy / ny)
        x = np.arange(nx) - nx // 2
        y = np.arange(ny) - ny // 2
        self.deapod = np.outer(kb_transform(y / self.gy, self.width, self.by),
                               kb_transform(x / self.gx, self.width, self.bx))
        traj = np.asarray(traj, dtype=np.float64)
        tx = traj[:, 0] * self.gx / (2.0 * math.pi)
        ty = traj[:, 1] * self.gy / (2.0 * math.pi)
        # the W grid points of each sample per axis and their weights
        self.mx, self.wx = self._neighbours(tx, self.gx, self.bx)
        self.my, self.wy = self._neighbours(ty, self.gy, self.by)

    def _neighbours(self, t, g, beta):
        w = self.width
        m0 = np.ceil(t - w / 2.0).astype(np.int64)
        m = m0[:, None] + np.arange(w + 1)[None, :]          # W + 1 covers ceil .. floor
        wt = kb_kernel(t[:, None] - m, w, beta)
        return np.mod(m, g), wt


def _to_grid(img, gy, gx):
    """Centred ny x nx image into a gy x gx grid at index (offset mod G)."""
    ny, nx = img.shape
    out = np.zeros((gy, gx), np.complex128)
    y = np.mod(np.arange(ny) - ny // 2, gy)
    x = np.mod(np.arange(nx) - nx // 2, gx)
    out[np.ix_(y, x)] = img
    return out


def _from_grid(grid, ny, nx):
    gy, gx = grid.shape
    y = np.mod(np.arange(ny) - ny // 2, gy)
    x = np.mod(np.arange(nx) - nx // 2, gx)
    return grid[np.ix_(y, x)]


def forward(image, smaps, plan):
    """d[g, k] ~ F(image), image [ny, nx], smaps [nc, ny, nx] -> [nc, nk]."""
    image = np.asarray(image, np.complex128)
    smaps = np.asarray(smaps, np.complex128)
    nc = smaps.shape[0]
    nk = plan.mx.shape[0]
    out = np.empty((nc, nk), np.complex128)
    for g in range(nc):
        u = np.fft.fft2(_to_grid(smaps[g] * image / plan.deapod, plan.gy, plan.gx))
        # sum over the W x W (here (W+1) x (W+1), zero weights outside) neighbours
        vals = u[plan.my[:, :, None], plan.mx[:, None, :]]
        out[g] = np.einsum("kyx,ky,kx->k", vals, plan.wy, plan.wx)
    return out


def adjoint(data, smaps, plan):
    """image ~ F^H(data), data [nc, nk] -> [ny, nx]: the exact adjoint of forward."""
    data = np.asarray(data, np.complex128)
    smaps = np.asarray(smaps, np.complex128)
    nc = smaps.shape[0]
    out = np.zeros((plan.ny, plan.nx), np.complex128)
    for g in range(nc):
        grid = np.zeros((plan.gy, plan.gx), np.complex128)
        contrib = data[g][:, None, None] * plan.wy[:, :, None] * plan.wx[:, None, :]
        np.add.at(grid, (np.broadcast_to(plan.my[:, :, None], contrib.shape),
                         np.broadcast_to(plan.mx[:, None, :], contrib.shape)), contrib)
        u = np.conj(np.fft.fft2(np.conj(grid)))               # unnormalised inverse DFT
        out += np.conj(smaps[g]) * _from_grid(u, plan.ny, plan.nx) / plan.deapod
    return out
