"""The overlapping multi-line layout (255 lines from 128 transmits, Sec. 3.3, Table 1) in the
CPU oracle: the layout's construction, lines without a transmit, the interpolation weights
(a constant channel signal stays constant through beamforming and combination) and a point
target between two transmits imaged on its own line."""
import numpy as np

import oracle
import synth


def combine64(y, g):
    return oracle.combine_lines(y, g.combine_src, g.combine_w)


def test_layout_construction():
    g = synth.config_overlap_2d()
    assert g.n_tx == 128 and g.n_out_lines == 255 and g.n_lines == 512
    np.testing.assert_allclose(np.asarray(g.combine_w, np.float64).sum(axis=1), 1.0)
    x_t = g.tx_origin[:, 0].astype(np.float64)
    for m in range(g.n_out_lines):
        ts = sorted({m // 2, (m + 1) // 2})
        srcs = [s for s in g.combine_src[m] if s >= 0]
        assert sorted(int(g.line_tx[s]) for s in srcs) == ts
        for s in srcs:  # every source beam lies on the output line's position
            assert abs(float(g.line_origin[s, 0]) - g.out_line_x[m]) < 1e-9
        # the output line sits on its transmit's axis (even) or half way between two (odd)
        assert abs(g.out_line_x[m] - np.mean(x_t[ts])) < 1e-9
    # unused slots carry no transmit and no weight
    unused = np.where(g.line_tx < 0)[0]
    assert len(unused) == 512 - (128 + 2 * 127)
    assert not np.isin(unused, g.combine_src).any()


def test_lines_without_transmit_are_zero():
    g = synth.config_overlap_2d(n_el=16, n_samples=256)
    rng = np.random.default_rng(0)
    rf = rng.integers(-3000, 3000, size=(1, g.n_tx, g.n_el, g.n_samples)).astype(np.int16)
    y = oracle.das(g, rf)
    unused = np.where(g.line_tx < 0)[0]
    assert np.all(y[0, unused] == 0.0)
    assert np.abs(y[0, g.line_tx >= 0]).max() > 0
    pix = np.stack([np.zeros(len(unused), int), unused, np.full(len(unused), 50)], 1)
    assert np.all(oracle.delay_gather(g, rf, pix) == 0.0)


def test_constant_signal_survives_beamforming_and_interpolation():
    """A channel signal equal to 1000 everywhere: every beam is 1000 wherever its whole aperture
    reads inside the record (normalised apodization), so every output line is 1000 there too
    (the interpolation weights sum to one)."""
    g = synth.config_overlap_2d(n_el=16, n_samples=512)
    rf = np.full((1, g.n_tx, g.n_el, g.n_samples), 1000, dtype=np.int16)
    y = oracle.das(g, rf)
    out = combine64(y, g)
    j = np.arange(20, 200)  # past the first samples, well before the end of the record
    np.testing.assert_allclose(out[0][:, j], 1000.0, rtol=0, atol=1e-9)


def test_point_between_two_transmits_is_imaged_on_its_line():
    g = synth.config_overlap_2d(n_el=32, n_samples=1024)
    m_star, j_star = 31, 300  # odd: half way between transmits 15 and 16
    slot = int(g.combine_src[m_star][0])
    pos = synth.phantom.pixel_position(g, slot, j_star)[None, :]
    rf = synth.rfsim.simulate_frame(g, pos, np.array([1.0]), seed=0, noise=False).numpy()
    env = oracle.envelope(combine64(oracle.das(g, rf), g)[0])
    m, j = np.unravel_index(np.argmax(env), env.shape)
    assert (m, j) == (m_star, j_star)
