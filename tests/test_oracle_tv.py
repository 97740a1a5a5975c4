"""Pins of the oracle's finite-difference transform and soft threshold
(Sec. III-A, eq. (9)-(10)) against dense matrices, closed forms and brute force."""
import math

import numpy as np
import pytest

from oracle import tv
from paper_2006_14080_amd import synth


def _dense(fn, n_in_shape):
    n = int(np.prod(n_in_shape))
    cols = []
    for t in range(n):
        e = np.zeros(n, np.complex128)
        e[t] = 1.0
        cols.append(np.asarray(fn(e.reshape(n_in_shape))).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("nx,ny", [(4, 4), (5, 3), (2, 7), (6, 1)])
def test_adjoint_is_conjugate_transpose(nx, ny):
    th = _dense(tv.tv_forward, (ny, nx))
    th_h = _dense(tv.tv_adjoint, (2, ny, nx))
    np.testing.assert_allclose(th_h, th.conj().T, atol=0)


def test_known_small_image():
    # Hand-computed periodic forward differences of [[1, 2, 4], [7, 11, 16]].
    v = np.array([[1, 2, 4], [7, 11, 16]], dtype=np.complex128)
    g = tv.tv_forward(v)
    np.testing.assert_array_equal(g[0].real, [[1, 2, -3], [4, 5, -9]])
    np.testing.assert_array_equal(g[1].real, [[6, 9, 12], [-6, -9, -12]])


@pytest.mark.parametrize("nx,ny", [(8, 8), (6, 5), (9, 4)])
def test_normal_spectrum_closed_form(nx, ny):
    # Theta^H Theta is the periodic 5-point Laplacian; its eigenvalues are
    # 4 sin^2(pi p / nx) + 4 sin^2(pi q / ny).
    m = _dense(lambda v: tv.tv_adjoint(tv.tv_forward(v)), (ny, nx))
    eig = np.sort(np.linalg.eigvalsh(m))
    ref = np.sort([4 * math.sin(math.pi * p / nx) ** 2 + 4 * math.sin(math.pi * q / ny) ** 2
                   for p in range(nx) for q in range(ny)])
    np.testing.assert_allclose(eig, ref, atol=1e-12)


def test_constant_image_has_zero_gradient():
    g = tv.tv_forward(np.full((5, 7), 2.5 - 1j))
    assert np.all(g == 0)


def test_adjoint_identity_random():
    a = synth.random_complex((9, 13), 1, np.complex128)
    g = synth.random_complex((2, 9, 13), 2, np.complex128)
    lhs = np.vdot(tv.tv_forward(a), g)
    rhs = np.vdot(a, tv.tv_adjoint(g))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_soft_threshold_real_cases():
    # Eq. (10) on real arguments with lambda/beta = 1.
    z = np.array([3.0, -3.0, 0.5, -0.5, 1.0, -1.0, 0.0, 1.25])
    out = tv.soft_threshold(z, 1.0)
    np.testing.assert_allclose(out.real, [2.0, -2.0, 0, 0, 0, 0, 0, 0.25], rtol=0, atol=1e-15)
    assert np.all(out.imag == 0)


def test_soft_threshold_is_the_prox_brute_force():
    # mu = argmin lam |mu| + (beta/2) |mu - v|^2, searched on a fine complex grid.
    rng = np.random.default_rng(3)
    lam, beta = 0.7, 2.0
    for _ in range(6):
        v = complex(*rng.uniform(-1.5, 1.5, 2))
        h = 2e-3
        re = np.arange(-2.0, 2.0, h)
        grid = re[None, :] + 1j * re[:, None]
        cost = lam * np.abs(grid) + 0.5 * beta * np.abs(grid - v) ** 2
        best = grid.ravel()[np.argmin(cost)]
        mu = tv.soft_threshold(np.array([v]), lam / beta)[0]
        assert abs(best - mu) <= 2 * h


def test_soft_threshold_subgradient_condition():
    rng = np.random.default_rng(4)
    v = rng.standard_normal(200) + 1j * rng.standard_normal(200)
    thr = 0.8
    mu = tv.soft_threshold(v, thr)
    big = np.abs(v) > thr
    # beta (mu - v) + lam mu/|mu| = 0 on the support (divide by beta).
    np.testing.assert_allclose(mu[big] - v[big] + thr * mu[big] / np.abs(mu[big]), 0, atol=1e-12)
    assert np.all(mu[~big] == 0)
