"""Pins of the oracle's NUDFT (eq. (1)-(2), Alg. 1, Alg. 3) against facts that
do not come from the oracle itself: NumPy's FFT on a Cartesian grid, scalar
brute force, the adjoint identity and linearity."""
import math

import numpy as np
import pytest

from oracle import nudft
from paper_2006_14080_amd import synth

SHAPES = [(8, 8), (8, 6), (5, 7), (4, 3), (3, 5)]


def _rand(shape, seed):
    return synth.random_complex(shape, seed, np.complex128)


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_cartesian_equals_centred_fft(nx, ny):
    # On the full Cartesian grid with unit sensitivity, eq. (1) with centred
    # coordinates is the centred DFT: fftshift(fft2(ifftshift(rho))).
    rho = _rand((ny, nx), 1)
    traj = synth.cartesian_trajectory(nx, ny)
    d = nudft.forward(rho, np.ones((1, ny, nx)), traj)
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(rho)))
    np.testing.assert_allclose(d[0].reshape(ny, nx), ref, rtol=0, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_cartesian_multicoil_fft(nx, ny):
    rho = _rand((ny, nx), 2)
    s = _rand((3, ny, nx), 3)
    traj = synth.cartesian_trajectory(nx, ny)
    d = nudft.forward(rho, s, traj)
    for g in range(3):
        ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(s[g] * rho)))
        np.testing.assert_allclose(d[g].reshape(ny, nx), ref, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("nx,ny", SHAPES)
def test_cartesian_adjoint_is_scaled_inverse(nx, ny):
    # Adjoint of the centred DFT is N times its inverse: F^H d = N ifft(d),
    # and F^H F = N I on the full grid.
    rho = _rand((ny, nx), 4)
    traj = synth.cartesian_trajectory(nx, ny)
    one = np.ones((1, ny, nx))
    dat = _rand((1, nx * ny), 5)
    back = nudft.adjoint(dat, one, traj)
    ref = nx * ny * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(dat[0].reshape(ny, nx))))
    np.testing.assert_allclose(back, ref, atol=1e-10 * np.abs(ref).max())
    np.testing.assert_allclose(nudft.adjoint(nudft.forward(rho, one, traj), one, traj),
                               nx * ny * rho, atol=1e-10 * nx * ny)


def _brute_forward(rho, s, traj):
    nc, ny, nx = s.shape
    out = np.zeros((nc, traj.shape[0]), np.complex128)
    for g in range(nc):
        for k in range(traj.shape[0]):
            acc = 0j
            for i in range(ny):
                for j in range(nx):
                    th = traj[k, 0] * (j - nx // 2) + traj[k, 1] * (i - ny // 2)
                    acc += s[g, i, j] * rho[i, j] * complex(math.cos(th), -math.sin(th))
            out[g, k] = acc
    return out


def _brute_adjoint(dat, s, traj):
    nc, ny, nx = s.shape
    out = np.zeros((ny, nx), np.complex128)
    for i in range(ny):
        for j in range(nx):
            acc = 0j
            for g in range(nc):
                for k in range(traj.shape[0]):
                    th = traj[k, 0] * (j - nx // 2) + traj[k, 1] * (i - ny // 2)
                    acc += s[g, i, j].conjugate() * dat[g, k] * complex(math.cos(th), math.sin(th))
            out[i, j] = acc
    return out


@pytest.mark.parametrize("nx,ny,nc,nk", [(4, 4, 2, 17), (5, 3, 3, 29), (8, 5, 1, 64), (3, 8, 2, 11)])
def test_brute_force_sums(nx, ny, nc, nk):
    rho = _rand((ny, nx), 6)
    s = _rand((nc, ny, nx), 7)
    traj = synth.random_trajectory(nk, 8)
    dat = _rand((nc, nk), 9)
    np.testing.assert_allclose(nudft.forward(rho, s, traj), _brute_forward(rho, s, traj),
                               rtol=0, atol=1e-11)
    np.testing.assert_allclose(nudft.adjoint(dat, s, traj), _brute_adjoint(dat, s, traj),
                               rtol=0, atol=1e-11)
    np.testing.assert_allclose(
        nudft.forward_samples(rho, s, traj, [0, nc - 1], [0, nk - 1]),
        _brute_forward(rho, s, traj)[[0, nc - 1], [0, nk - 1]], atol=1e-11)
    np.testing.assert_allclose(
        nudft.adjoint_pixels(dat, s, traj, [0, ny - 1], [nx - 1, 0]),
        _brute_adjoint(dat, s, traj)[[0, ny - 1], [nx - 1, 0]], atol=1e-11)


@pytest.mark.parametrize("nx,ny,nc,nk", [(16, 12, 3, 300), (32, 32, 4, 1024), (7, 9, 2, 50)])
def test_adjoint_identity(nx, ny, nc, nk):
    rho = _rand((ny, nx), 10)
    s = _rand((nc, ny, nx), 11)
    traj = synth.random_trajectory(nk, 12)
    dat = _rand((nc, nk), 13)
    lhs = np.vdot(nudft.forward(rho, s, traj), dat)
    rhs = np.vdot(rho, nudft.adjoint(dat, s, traj))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) * 10


def test_linearity():
    nx, ny, nc, nk = 12, 10, 2, 80
    s = _rand((nc, ny, nx), 14)
    traj = synth.random_trajectory(nk, 15)
    a, b = _rand((ny, nx), 16), _rand((ny, nx), 17)
    ca, cb = 0.3 - 1.2j, -2.0 + 0.5j
    lhs = nudft.forward(ca * a + cb * b, s, traj)
    rhs = ca * nudft.forward(a, s, traj) + cb * nudft.forward(b, s, traj)
    np.testing.assert_allclose(lhs, rhs, atol=1e-11)


def test_axis_pairing_single_frequency():
    # A plane wave exp(+i w0 x) (x along the fast axis) is detected at the sample
    # whose column-0 frequency is w0 and column-1 frequency is 0; swapping the
    # columns of the trajectory moves the peak.
    nx, ny = 16, 8
    w0 = 2 * math.pi * 3 / nx
    x = nudft.grid_coords(nx)[None, :]
    rho = np.exp(1j * w0 * x) * np.ones((ny, 1))
    traj = np.array([[w0, 0.0], [0.0, w0]])
    d = nudft.forward(rho, np.ones((1, ny, nx)), traj)
    assert abs(d[0, 0] - nx * ny) < 1e-9
    assert abs(d[0, 1]) < 1e-9
