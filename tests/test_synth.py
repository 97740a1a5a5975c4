"""Seeded generators: reproducibility, ranges and structure of the inputs."""
import math

import numpy as np

from paper_2006_14080_amd import synth


def test_seeds_reproduce():
    a = synth.make_problem(synth.ADMM32)
    b = synth.make_problem(synth.ADMM32)
    for x, y in [(a.truth, b.truth), (a.smaps, b.smaps), (a.traj, b.traj), (a.noise, b.noise)]:
        assert np.array_equal(x, y)
    c = synth.ellipse_phantom(32, 32, 102)
    assert not np.array_equal(a.truth[0], c)


def test_shapes_and_dtypes():
    p = synth.make_problem(synth.ADMM32)
    wl = synth.ADMM32
    assert p.truth.shape == (1, 32, 32) and p.truth.dtype == np.complex64
    assert p.smaps.shape == (4, 32, 32) and p.smaps.dtype == np.complex64
    assert p.traj.shape == (wl.nk, 2) and p.traj.dtype == np.float64
    assert p.noise.shape == (1, 4, wl.nk)
    assert wl.nk == 1024 and synth.ADMM256.nk == 32768 and synth.SLICES384.nk == 98304


def test_trajectory_range_and_golden_angle():
    t = synth.radial_trajectory(16, 64)
    r = np.hypot(t[:, 0], t[:, 1])
    assert r.max() <= math.pi + 1e-12
    assert np.all(t >= -math.pi - 1e-12) and np.all(t <= math.pi + 1e-12)
    # readout 0 of every spoke sits at radius pi, the centre sample at radius 0
    assert np.allclose(r[0::64], math.pi) and np.allclose(r[32::64], 0.0)
    ang = math.atan2(t[64 + 63, 1], t[64 + 63, 0])
    assert abs(ang - synth.GOLDEN_ANGLE) < 1e-12


def test_coil_maps_rotate_with_coil_index():
    s = synth.coil_maps(16, 16, 4)
    mag = np.abs(s)
    # coil 0 sits at +x (right edge), coil 2 at -x (left edge)
    assert mag[0, 8, 15] > mag[0, 8, 0]
    assert mag[2, 8, 0] > mag[2, 8, 15]
    # coil 1 (a quarter turn on) sits at +y (last rows), coil 3 at -y
    assert mag[1, 15, 8] > mag[1, 0, 8] and mag[3, 0, 8] > mag[3, 15, 8]
    # each coil carries the constant phase exp(i phi)
    np.testing.assert_allclose(np.angle(s[1]), math.pi / 2, atol=1e-6)


def test_phantom_is_piecewise_constant_and_real():
    p = synth.ellipse_phantom(64, 48, 7)
    assert np.all(p.imag == 0) and p.real.min() >= 0
    assert len(np.unique(p.real)) < 200


def test_request_stream_is_seeded_and_poisson():
    r1 = synth.request_stream(200)
    r2 = synth.request_stream(200)
    assert [q.wl for q in r1] == [q.wl for q in r2]
    gaps = np.diff([0.0] + [q.arrival for q in r1])
    assert 0.03 < gaps.mean() < 0.07
    assert {q.wl.nx for q in r1} == {128, 256, 384}
    assert all(4 <= q.wl.nc <= 32 and 32 <= q.wl.n_spokes <= 128 for q in r1)
    assert all(q.wl.n_readout == 2 * q.wl.nx for q in r1)
