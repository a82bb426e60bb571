"""Plane-wave transmits (infinite focus), diverging waves (a virtual source behind the array)
and coherent compounding in the CPU oracle, pinned to closed forms, brute force and the
binary32 rule (plane-wave imaging, Sec. 2)."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.test_oracle_das import custom_geom, _brute_das


def planewave_geom(theta_deg, el_x, line_x, **kw):
    g = custom_geom(el_x=el_x, line_x=line_x, tx_x=[0.0], line_tx=np.zeros(len(line_x), np.int32), **kw)
    th = math.radians(theta_deg)
    g.tx_dir = np.float32([[math.sin(th), 0.0, math.cos(th)]])
    g.tx_focus = np.float32([np.inf])
    return g


def test_unsteered_plane_wave_under_the_element_is_twice_depth():
    """theta = 0, element under the line: the wave reaches depth r after r / c and returns
    after another r / c, so tau = 2 r fs / c = j (depth_step 1, c = 1500, fs = 37.5 MHz)."""
    g = planewave_geom(0.0, el_x=[0.0, 1e-3], line_x=[0.0, 1e-3])
    js = np.array([1, 200, 511])
    for l in (0, 1):
        tau = oracle.tau64(g, np.stack([np.full(js.size, l), js], 1))
        np.testing.assert_allclose(tau[:, l], js, atol=1e-9)
        i0, phi, _, _ = oracle.tof32(g, np.stack([np.full(js.size, l), js], 1))
        assert np.all(i0[:, l] == js) and np.all(phi[:, l] == 0.0)


def test_steered_plane_wave_hand_computed():
    """theta = 30 deg, pixel 4 mm deep on the line through x = 0, element at x = 3 mm: transmit
    path 4 mm cos 30 deg = 3.4641016 mm, receive path 5 mm, tau = 8.4641016 mm fs / c =
    211.602540 samples."""
    g = planewave_geom(30.0, el_x=[0.0, 3e-3], line_x=[0.0])
    j = 200
    tau = oracle.tau64(g, [[0, j]])[0]
    assert tau[1] == pytest.approx(211.60254037844386, abs=1e-6)   # (4 cos 30 + 5) mm * 25 / mm
    assert tau[0] == pytest.approx(100.0 * (4 * math.sqrt(3) / 2 + 4) * 0.25, abs=1e-6)
    i0, phi, _, _ = oracle.tof32(g, [[0, j]])
    assert i0[0, 1] + phi[0, 1] == pytest.approx(211.6025404, abs=1e-4)


def test_binary32_rule_tracks_float64_for_plane_waves():
    g = synth.config_planewave_2d(n_samples=2048, lines=64)
    rng = np.random.default_rng(3)
    pix = np.stack([rng.integers(0, g.n_lines, 3000), rng.integers(0, g.n_depth, 3000)], 1)
    tau = oracle.tau64(g, pix)
    i0, phi, act, val = oracle.tof32(g, pix)
    err = np.abs((i0 + phi) - tau)[act]
    assert err.max() < 1e-4


def test_plane_wave_das_brute_force():
    g = planewave_geom(12.0, el_x=np.arange(6) * 0.3e-3 - 0.75e-3, line_x=[-0.3e-3, 0.0, 0.45e-3],
                       n_samples=96, n_depth=40, depth_step=2)
    g.tx_dir = np.float32([[math.sin(math.radians(12.0)), 0.0, math.cos(math.radians(12.0))]])
    rng = np.random.default_rng(5)
    rf = rng.integers(-3000, 3000, size=(1, 1, 6, 96)).astype(np.int16)
    y = oracle.das(g, rf)

    def brute(l, j):
        # the brute force of the focused case with the plane-wave transmit path
        t = 0
        o = g.line_origin[l].astype(float)
        r = (g.depth_start + g.depth_step * j) * g.c / (2 * g.fs)
        p = o + r * np.array([0.0, 0.0, 1.0])
        dt = g.tx_dir[t].astype(float)
        dt /= math.sqrt(dt @ dt)
        ctx = float(p @ dt)
        _, _, act, val = oracle.tof32(g, [[l, j]])
        num = den = 0.0
        for e in range(g.n_el):
            if not act[0, e]:
                continue
            dx = float(g.el_pos[e, 0]) - float(o[0])
            w = 1.0 if r == 0 else 0.5 + 0.5 * math.cos(2 * math.pi * dx * g.f_number / r)
            den += w
            if not val[0, e]:
                continue
            ev = g.el_pos[e].astype(float)
            tau = g.fs * (ctx + math.sqrt(float((ev - p) @ (ev - p)))) / g.c
            i = int(math.floor(tau))
            ph = tau - i
            tr = rf[0, t, e].astype(float)
            num += w * ((1 - ph) * tr[i] + ph * tr[i + 1])
        return num / den if den > 0 else 0.0

    for l in range(3):
        for j in range(40):
            assert y[0, l, j] == pytest.approx(brute(l, j), abs=1e-9)


def test_plane_waves_image_a_point_at_its_pixel():
    """A point target simulated with 5 plane waves: the compounded beamformed frame's envelope
    peaks on the target's pixel."""
    g = synth.config_planewave_2d(n_angles=5, n_samples=1024, lines=64, scan_n=(64, 64))
    l_star, j_star = 30, 300
    pos = synth.phantom.pixel_position(g, l_star, j_star)[None, :]
    rf = synth.rfsim.simulate_frame(g, pos, np.array([1.0]), seed=0, noise=False).numpy()
    y = oracle.das(g, rf)[0].reshape(5, 64, g.n_depth).mean(axis=0)
    env = oracle.envelope(y)
    l, j = np.unravel_index(np.argmax(env), env.shape)
    assert (l, j) == (l_star, j_star)


def divergingwave_geom(theta_deg, behind, el_x, line_x, **kw):
    g = custom_geom(el_x=el_x, line_x=line_x, tx_x=[0.0], line_tx=np.zeros(len(line_x), np.int32), **kw)
    th = math.radians(theta_deg)
    g.tx_dir = np.float32([[math.sin(th), 0.0, math.cos(th)]])
    g.tx_focus = np.float32([-behind])
    return g


def test_diverging_wave_hand_computed():
    """Virtual source 5 mm behind the array centre, pixel 4 mm deep on the line through
    x = 3 mm, element under the pixel: the wave leaves the source at -|F| / c, so the transmit
    path is sqrt(3^2 + 9^2) - 5 = 4.4868330 mm, the receive path 4 mm, tau = 8.4868330 mm x
    25 samples/mm = 212.170825 (c = 1500, fs = 37.5 MHz).  On the axis through the source the
    transmit path is the depth itself."""
    g = divergingwave_geom(0.0, 5e-3, el_x=[0.0, 3e-3], line_x=[0.0, 3e-3])
    tau = oracle.tau64(g, [[1, 200], [0, 200]])
    assert tau[0, 1] == pytest.approx(25.0 * (math.sqrt(90.0) - 5.0 + 4.0), abs=1e-6)
    assert tau[1, 0] == pytest.approx(200.0, abs=1e-9)
    i0, phi, act, _ = oracle.tof32(g, [[1, 200], [0, 200]])
    assert act[0, 1] and i0[0, 1] + phi[0, 1] == pytest.approx(212.1708245, abs=1e-4)
    assert i0[1, 0] == 200 and phi[1, 0] == 0.0


def test_diverging_wave_arrival_is_later_than_plane_wave_off_axis():
    """Off the source's axis a diverging wave arrives later than the unsteered plane wave
    (the spherical front lags the flat one by sqrt(x^2 + (r + d)^2) - (r + d)), and the lag
    shrinks towards the plane wave as the source moves back."""
    lags = []
    for d in (2e-3, 10e-3, 100e-3):
        gd = divergingwave_geom(0.0, d, el_x=[6e-3], line_x=[6e-3])
        gp = planewave_geom(0.0, el_x=[6e-3], line_x=[6e-3])
        lag = oracle.tau64(gd, [[0, 300]])[0, 0] - oracle.tau64(gp, [[0, 300]])[0, 0]
        r = 6e-3  # j = 300 at 25 samples/mm and depth_step 1 is 6 mm
        assert lag == pytest.approx(25e3 * (math.hypot(6e-3, r + d) - (r + d)), abs=1e-6)
        lags.append(lag)
    assert lags[0] > lags[1] > lags[2] > 0


def test_binary32_rule_tracks_float64_for_diverging_waves():
    g = synth.config_planewave_2d(n_samples=2048, lines=64, focus=-20e-3, max_angle_deg=20.0)
    rng = np.random.default_rng(4)
    pix = np.stack([rng.integers(0, g.n_lines, 3000), rng.integers(0, g.n_depth, 3000)], 1)
    tau = oracle.tau64(g, pix)
    i0, phi, act, val = oracle.tof32(g, pix)
    err = np.abs((i0 + phi) - tau)[act]
    assert err.max() < 1e-4


def test_diverging_waves_image_a_point_at_its_pixel():
    g = synth.config_planewave_2d(n_angles=5, n_samples=1024, lines=64, scan_n=(64, 64), focus=-15e-3,
                                  max_angle_deg=15.0)
    l_star, j_star = 12, 350
    pos = synth.phantom.pixel_position(g, l_star, j_star)[None, :]
    rf = synth.rfsim.simulate_frame(g, pos, np.array([1.0]), seed=0, noise=False).numpy()
    y = oracle.das(g, rf)[0].reshape(5, 64, g.n_depth).mean(axis=0)
    env = oracle.envelope(y)
    l, j = np.unravel_index(np.argmax(env), env.shape)
    assert (l, j) == (l_star, j_star)
