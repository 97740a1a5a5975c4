"""Pins of the oracle's NUFFT (oracle/nufft.py), the approximation of the
NUDFT by Kaiser-Bessel gridding and an oversampled FFT (the operator of the
paper's comparison systems, Sec. VII / Table II).

* the closed-form Fourier transform of the kernel equals a numerical
  integral of the kernel (so the deapodisation divides by the right thing);
* the NUFFT approaches the exact NUDFT (oracle.nudft) as the kernel widens,
  each extra grid point of width gaining close to an order of magnitude, and
  stays under the stated bounds (width 6: 1e-5, width 7: 1e-6 relative);
* the adjoint is the exact adjoint of the forward;
* a single pixel has the same NUFFT as the NUDFT's plane wave, sample by
  sample, within the bound.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import nudft, nufft
from paper_2006_14080_amd import synth

BOUND = {6: 1e-5, 7: 1e-6}


@pytest.mark.parametrize("width,sigma", [(4, 2.0), (6, 2.0), (7, 2.5), (8, 2.0)])
def test_kernel_transform_closed_form(width, sigma):
    beta = nufft.kb_beta(width, sigma)
    for f in [0.0, 0.05, 0.13, 0.25, 0.4]:
        num, _ = integrate.quad(lambda u: float(nufft.kb_kernel(np.array([u]), width, beta)[0]) *
                                math.cos(2 * math.pi * u * f), -width / 2, width / 2, limit=200)
        got = float(nufft.kb_transform(np.array([f]), width, beta)[0])
        assert abs(got - num) <= 1e-9 * abs(num)


def _problem(nx=40, ny=28, nc=3, spokes=20, nr=96):
    img = synth.ellipse_phantom(nx, ny, 9).astype(np.complex128)
    sm = synth.coil_maps(nx, ny, nc)
    traj = synth.radial_trajectory(spokes, nr)
    return img, sm, traj


def test_error_falls_with_kernel_width():
    img, sm, traj = _problem()
    ref = nudft.forward(img, sm, traj)
    errs = []
    for w in range(4, 9):
        f = nufft.forward(img, sm, nufft.Plan(img.shape[1], img.shape[0], traj, width=w))
        errs.append(np.linalg.norm(f - ref) / np.linalg.norm(ref))
    for a, b in zip(errs, errs[1:]):
        assert b < a / 4
    assert errs[0] < 1e-2


@pytest.mark.parametrize("width", [6, 7])
def test_forward_and_adjoint_within_bound(width):
    img, sm, traj = _problem()
    p = nufft.Plan(img.shape[1], img.shape[0], traj, width=width)
    ref = nudft.forward(img, sm, traj)
    assert np.linalg.norm(nufft.forward(img, sm, p) - ref) <= BOUND[width] * np.linalg.norm(ref)
    dat = synth.random_complex((sm.shape[0], traj.shape[0]), 4, np.complex128)
    refa = nudft.adjoint(dat, sm, traj)
    assert np.linalg.norm(nufft.adjoint(dat, sm, p) - refa) <= BOUND[width] * np.linalg.norm(refa)


@pytest.mark.parametrize("nx,ny,sigma", [(32, 32, 2.0), (24, 40, 2.0), (21, 17, 1.5)])
def test_adjoint_identity(nx, ny, sigma):
    sm = synth.random_complex((2, ny, nx), 5, np.complex128)
    traj = synth.random_trajectory(300, 6)
    p = nufft.Plan(nx, ny, traj, width=6, sigma=sigma)
    x = synth.random_complex((ny, nx), 7, np.complex128)
    y = synth.random_complex((2, 300), 8, np.complex128)
    lhs = np.vdot(nufft.forward(x, sm, p), y)
    rhs = np.vdot(x, nufft.adjoint(y, sm, p))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_single_pixel_is_a_plane_wave():
    nx, ny = 32, 24
    img = np.zeros((ny, nx), np.complex128)
    j, i = 7, 19
    img[i, j] = 1.0
    traj = synth.random_trajectory(200, 10)
    p = nufft.Plan(nx, ny, traj, width=7)
    got = nufft.forward(img, np.ones((1, ny, nx)), p)[0]
    want = np.exp(-1j * (traj[:, 0] * (j - nx // 2) + traj[:, 1] * (i - ny // 2)))
    assert np.max(np.abs(got - want)) <= 1e-6
