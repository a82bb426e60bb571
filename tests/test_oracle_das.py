"""Pins of the CPU oracle's delays and delay-and-sum against closed forms, special cases and
invariants (receive beamforming, Sec. 1 pipeline list / Sec. 2 method list)."""
import math

import numpy as np
import pytest

import oracle
import synth
from synth.geometry import Geometry, HANN, RECT, linear_array


def custom_geom(el_x, line_x, tx_x=None, line_tx=None, focus=30e-3, c=1500.0, fs=37.5e6,
                n_samples=1024, f_number=1.0, window=HANN, depth_step=1, n_depth=None,
                array_dims=1, el_y=None):
    el_x = np.asarray(el_x, np.float64)
    n_el = el_x.size
    el = np.zeros((n_el, 3), np.float32)
    el[:, 0] = el_x
    if el_y is not None:
        el[:, 1] = el_y
    line_x = np.asarray(line_x, np.float64)
    nl = line_x.size
    lo = np.zeros((nl, 3), np.float32)
    lo[:, 0] = line_x
    ld = np.tile(np.float32([0, 0, 1]), (nl, 1))
    if tx_x is None:
        to, td = lo.copy(), ld.copy()
        lt = np.arange(nl, dtype=np.int32)
    else:
        tx_x = np.asarray(tx_x, np.float64)
        to = np.zeros((tx_x.size, 3), np.float32)
        to[:, 0] = tx_x
        td = np.tile(np.float32([0, 0, 1]), (tx_x.size, 1))
        lt = np.asarray(line_tx, np.int32)
    return Geometry(name="custom", el_pos=el, tx_origin=to, tx_dir=td,
                    tx_focus=np.full(to.shape[0], focus, np.float32), line_origin=lo, line_dir=ld,
                    line_tx=lt, array_dims=array_dims, c=float(np.float32(c)), fs=float(np.float32(fs)),
                    t0=0.0, n_samples=n_samples, depth_start=0, depth_step=depth_step,
                    n_depth=n_depth or n_samples // depth_step, f_number=float(np.float32(f_number)),
                    window=window, f0=5e6)


# ------------------------------------------------------------------ delays

def test_delay_on_axis_element_is_twice_depth():
    """Element at the line origin, pixel on the transmit axis: tau = 2 r fs / c = j0 + m j."""
    g = synth.config_small_2d()
    js = np.array([1, 100, 555, 1023])
    for l in (0, 17, 63):
        pix = np.stack([np.full(js.size, l), js], 1)
        tau = oracle.tau64(g, pix)
        np.testing.assert_allclose(tau[:, l], 2.0 * js, rtol=0, atol=1e-9)
        i0, phi, act, val = oracle.tof32(g, pix)
        assert np.all(i0[:, l] == 2 * js) and np.all(phi[:, l] == 0.0)


def test_delay_3_4_5_triangle():
    """Element 3 mm beside a line, pixel 4 mm deep on it (before the focus): transmit path 4 mm,
    receive path 5 mm, so tau = 9 mm * fs / c = 225 samples (c = 1500, fs = 37.5 MHz)."""
    g = custom_geom(el_x=[0.0, 3e-3], line_x=[0.0])
    j = 200                                   # depth = 200 * c / (2 fs) = 4 mm
    assert abs(g.depth_of(j) - 4e-3) < 1e-15
    tau = oracle.tau64(g, [[0, j]])
    np.testing.assert_allclose(tau[0], [200.0, 225.0], atol=1e-9)
    i0, phi, act, val = oracle.tof32(g, [[0, j]])
    assert i0[0, 1] + phi[0, 1] == pytest.approx(225.0, abs=1e-4)


def test_delay_at_and_beyond_focus():
    """Pixel at the focal point: T_tx = F / c.  Pixel off the transmit axis beyond the focus
    (multi-line receive): T_tx = (F + |p - focus|) / c."""
    F = 30e-3
    g = custom_geom(el_x=[0.0, 2e-3], line_x=[0.0, 0.6e-3], tx_x=[0.0], line_tx=[0, 0], focus=F,
                    n_samples=4096)
    jF = 1500                                 # 1500 * 2e-5 = 30 mm
    tau = oracle.tau64(g, [[0, jF], [1, 2000]])
    assert tau[0, 0] == pytest.approx(jF, abs=1e-9)     # depth step 1: tau = j on axis
    # positions are binary32 inputs: use their exact values
    xl, xe, F = (float(np.float32(v)) for v in (0.6e-3, 2e-3, F))
    r = 2000 * 2e-5
    ttx = F + math.hypot(xl, r - F)
    trx = math.hypot(xe - xl, r)
    assert tau[1, 1] == pytest.approx((ttx + trx) * 37.5e6 / 1500.0, abs=1e-9)
    # before the focus the converging wave reaches the pixel before the focal time
    r2 = 500 * 2e-5
    tau2 = oracle.tau64(g, [[1, 500]])
    ttx2 = F - math.hypot(xl, r2 - F)
    assert tau2[0, 0] == pytest.approx((ttx2 + math.hypot(xl, r2)) * 25000.0, abs=1e-9)


@pytest.mark.parametrize("cfg", ["small", "multiline"])
def test_binary32_delay_rule_tracks_float64(cfg):
    """The binary32 rearranged delay agrees with the direct float64 delay to ~1e-4 samples, and
    their integer parts differ only where tau is within that distance of an integer."""
    g = synth.config_small_2d() if cfg == "small" else synth.config_multiline_2d()
    rng = np.random.default_rng(5)
    pix = np.stack([rng.integers(0, g.n_lines, 3000), rng.integers(0, g.n_depth, 3000)], 1)
    tau = oracle.tau64(g, pix)
    i0, phi, act, val = oracle.tof32(g, pix)
    t32 = i0.astype(np.float64) + phi.astype(np.float64)
    err = np.abs(t32 - tau)
    # inside the aperture the rearranged binary32 rule stays within 1e-4 samples; outside it
    # (large lateral offsets at shallow depth, never summed) within 5e-4
    assert err[act].max() < 1e-4, err[act].max()
    assert np.sqrt(np.mean(err[act] ** 2)) < 1e-5
    assert err.max() < 5e-4
    diff = i0 != np.floor(tau)
    near = np.abs(tau - np.round(tau)) < np.where(act, 1e-4, 5e-4)
    assert np.all(near[diff])


def test_binary32_delay_rule_3d_steered():
    g = synth.config_volume_3d()
    rng = np.random.default_rng(9)
    pix = np.stack([rng.integers(0, g.n_lines, 200), rng.integers(0, g.n_depth, 200)], 1)
    tau = oracle.tau64(g, pix)
    i0, phi, act, val = oracle.tof32(g, pix)
    err = np.abs(i0 + phi.astype(np.float64) - tau)
    assert err[act].max() < 1e-4, err.max()


def test_aperture_grows_with_depth():
    """F# = 1: the active elements at depth r are those within r/2 of the line; their count
    is the number of pitch positions inside that width, by hand."""
    g = synth.config_small_2d()
    l = 31
    js = np.array([0, 50, 300, 350, 1023])
    i0, phi, act, val = oracle.tof32(g, np.stack([np.full(js.size, l), js], 1))
    lx = g.line_origin[l, 0]
    for k, j in enumerate(js):
        r = np.float32(np.float32(2 * j) * np.float32(g.c / (2 * g.fs)))
        want = np.abs(g.el_pos[:, 0] - lx) * np.float32(2.0) <= r
        assert np.array_equal(act[k], want)
    n_act = act.sum(1)
    assert n_act[0] == 1 and np.all(np.diff(n_act) >= 0)
    # j = 350 -> 700 samples * c/(2 fs) = 13.475 mm deep -> half-aperture 6.74 mm = 22.46 pitches
    assert n_act[3] == 1 + 22 + 22
    assert n_act[4] == 64


# ------------------------------------------------------------------ delay and sum

def test_single_channel_rect_equals_interpolation():
    """Only the element under the line is active (huge F#), rectangular weight: DAS is that
    channel linearly interpolated at its delay (numpy.interp)."""
    g = synth.config_small_2d()
    g.f_number = 1e6
    g.window = RECT
    rng = np.random.default_rng(3)
    rf = rng.integers(-2000, 2000, size=(1, g.n_tx, g.n_el, g.n_samples)).astype(np.int16)
    l = 20
    js = np.arange(1, g.n_depth, 37)
    pix = np.stack([np.zeros_like(js), np.full(js.size, l), js], 1)
    y = oracle.das(g, rf, pix)
    tau = oracle.tau64(g, pix[:, 1:])[:, l]
    want = np.interp(tau, np.arange(g.n_samples), rf[0, l, l].astype(np.float64))
    want[tau > g.n_samples - 1] = 0.0
    np.testing.assert_allclose(y, want, rtol=0, atol=1e-9)


def test_hann_weights_closed_form():
    """Five elements at -2p..2p around the line; depth and F# chosen so the aperture is 4p wide:
    Hann weights are 0, 1/2, 1, 1/2, 0 (the outer two sit on the aperture edge).  With each
    channel constant, DAS = (a1/2 + a2 + a3/2) / 2."""
    p = 0.3e-3
    g = custom_geom(el_x=np.arange(-2, 3) * p, line_x=[0.0], n_samples=2048)
    j = 1000
    r = g.depth_of(j)
    g.f_number = float(np.float32(r / (4 * p)))
    vals = np.array([700, -300, 1000, 200, -900], np.int16)
    rf = np.broadcast_to(vals[None, None, :, None], (1, 1, 5, g.n_samples)).copy()
    y = oracle.das(g, rf, [[0, 0, j]])[0]
    assert y == pytest.approx((0.5 * -300 + 1000 + 0.5 * 200) / 2.0, rel=1e-6)


def test_constant_channels_give_constant_output():
    """Every sample equal to K: wherever all active delays fall inside the record, DAS = K."""
    g = synth.config_small_2d()
    rf = np.full((1, g.n_tx, g.n_el, g.n_samples), 1234, np.int16)
    js = np.arange(1, 900, 7)
    pix = np.stack([np.zeros_like(js), np.full(js.size, 40), js], 1)
    y = oracle.das(g, rf, pix)
    np.testing.assert_allclose(y, 1234.0, rtol=1e-12)


def test_das_is_linear():
    g = synth.config_small_2d()
    rng = np.random.default_rng(11)
    a = rng.integers(-1000, 1000, size=(1, g.n_tx, g.n_el, g.n_samples)).astype(np.int16)
    b = rng.integers(-1000, 1000, size=(1, g.n_tx, g.n_el, g.n_samples)).astype(np.int16)
    pix = np.stack([np.zeros(500, int), rng.integers(0, 64, 500), rng.integers(0, 1024, 500)], 1)
    ya, yb = oracle.das(g, a, pix), oracle.das(g, b, pix)
    yab = oracle.das(g, (a + b).astype(np.int16), pix)
    np.testing.assert_allclose(yab, ya + yb, rtol=0, atol=1e-9 * np.abs(ya).max())
    y3 = oracle.das(g, (3 * a).astype(np.int16), pix)
    np.testing.assert_allclose(y3, 3 * ya, rtol=0, atol=1e-9 * np.abs(ya).max())


def _brute_das(g, rf, f, l, j):
    """Independent float64 nested loops straight from the geometry (no rearrangement)."""
    t = int(g.line_tx[l])
    o = g.line_origin[l].astype(float)
    d = g.line_dir[l].astype(float)
    d /= math.sqrt(d @ d)
    ot = g.tx_origin[t].astype(float)
    dt = g.tx_dir[t].astype(float)
    dt /= math.sqrt(dt @ dt)
    F = float(g.tx_focus[t])
    r = (g.depth_start + g.depth_step * j) * g.c / (2 * g.fs)
    p = o + r * d
    focus = ot + F * dt
    along = float((p - ot) @ dt)
    dist_f = math.sqrt(float((p - focus) @ (p - focus)))
    ctx = F + dist_f if along >= F else F - dist_f
    _, _, act, val = oracle.tof32(g, [[l, j]])
    num = den = 0.0
    for e in range(g.n_el):
        if not act[0, e]:
            continue
        dx = float(g.el_pos[e, 0]) - float(o[0])
        w = 1.0 if r == 0 else (0.5 + 0.5 * math.cos(2 * math.pi * dx * g.f_number / r)
                                if g.window == HANN else 1.0)
        den += w
        if not val[0, e]:
            continue
        ev = g.el_pos[e].astype(float)
        tau = g.fs * (ctx + math.sqrt(float((ev - p) @ (ev - p)))) / g.c
        tau = min(max(tau, 0.0), g.n_samples - 1.0)
        i = int(math.floor(tau))
        ph = tau - i
        tr = rf[f, t, e].astype(float)
        s = tr[i] if i >= g.n_samples - 1 else (1 - ph) * tr[i] + ph * tr[i + 1]
        num += w * s
    return num / den if den > 0 else 0.0


def test_das_brute_force_tiny():
    g = synth.config_tiny(n_el=4, n_tx=2, lines_per_tx=3, n_samples=32)
    rng = np.random.default_rng(1)
    rf = rng.integers(-3000, 3000, size=(2, g.n_tx, g.n_el, g.n_samples)).astype(np.int16)
    y = oracle.das(g, rf)
    for f in range(2):
        for l in range(g.n_lines):
            for j in range(g.n_depth):
                assert y[f, l, j] == pytest.approx(_brute_das(g, rf, f, l, j), abs=1e-9)


def test_point_scatterer_focuses_on_its_pixel():
    """A single noiseless point target placed on an output pixel, away from the focus and off
    the centre: every active channel, once delayed, reads the pulse peak, and the envelope of
    the beamformed frame peaks exactly on that pixel."""
    g = synth.config_small_2d()
    l_star, j_star = 21, 700
    pos = synth.phantom.pixel_position(g, l_star, j_star)[None, :]
    rf = synth.rfsim.simulate_frame(g, pos, np.array([1.0]), seed=0, noise=False).numpy()
    x = oracle.delay_gather(g, rf, [[0, l_star, j_star]])[0]
    _, _, act, _ = oracle.tof32(g, [[l_star, j_star]])
    xa = x[act[0]]
    assert xa.min() > 0.97 * 30000 * 0.9 and xa.max() <= 30000.5
    y = oracle.das(g, rf)[0]
    env = oracle.envelope(y)
    l, j = np.unravel_index(np.argmax(env), env.shape)
    assert (l, j) == (l_star, j_star)
