"""Host-side image measures of the learned-apodization comparison, on closed forms."""
import numpy as np

from paper_1711_06127_amd import learned as L


def test_psf_width_of_gaussian_profile():
    # envelope exp(-x^2 / (2 s^2)) has its -6 dB (half amplitude) width 2 s sqrt(2 ln 2)
    lx = np.arange(200) * 0.1e-3
    s = 0.4e-3
    env = np.zeros((200, 50))
    for (l0, j0) in [(60, 10), (140, 30)]:
        env[:, j0] += np.exp(-((lx - lx[l0]) ** 2) / (2 * s * s))
    w = L.psf_widths(env, lx, [(60, 10), (140, 30)])
    exact = 2 * s * np.sqrt(2 * np.log(2))
    assert np.allclose(w, exact, rtol=0.02)


def test_psf_width_at_the_edge_is_bounded():
    lx = np.arange(20) * 1e-3
    env = np.ones((20, 5))
    w = L.psf_widths(env, lx, [(10, 2)])
    assert w[0] == lx[-1] - lx[0]


def test_cnr_of_two_constant_regions_with_known_spread():
    rng = np.random.default_rng(0)
    lx = np.linspace(-10e-3, 10e-3, 201)
    z = np.linspace(0, 40e-3, 401)
    X, Z = np.meshgrid(lx, z, indexing="ij")
    env = 1.0 + 0.1 * rng.standard_normal(X.shape)
    inside = (X ** 2 + (Z - 20e-3) ** 2) <= (4e-3) ** 2
    env[inside] = 0.2 + 0.05 * rng.standard_normal(inside.sum())
    c = L.cnr(env, lx, z, [(0.0, 20e-3, 4e-3)])
    exact = 0.8 / np.sqrt(0.1 ** 2 + 0.05 ** 2)
    assert abs(c[0] - exact) / exact < 0.05


def test_pixel_lists():
    p = L.frame_pixels(3, 4, 0, "cpu")
    assert p.shape == (12, 3)
    assert p[5].tolist() == [0, 1, 1]
    import torch
    gen = torch.Generator()
    gen.manual_seed(0)
    r = L.random_pixels(gen, 1000, 2, 5, 7, 3, "cpu")
    assert r[:, 0].max() <= 1 and r[:, 1].max() <= 4 and r[:, 2].min() >= 3 and r[:, 2].max() <= 6


def test_initial_network_is_near_uniform():
    p = L.init_params(0, 128)
    assert p["b4"][0] == np.float32(1 / 128)
    assert np.abs(p["W4"]).max() <= 1e-3 * np.sqrt(6 / 160) + 1e-9


def test_auxiliary_lines_take_the_nearest_transmit():
    import synth
    g = synth.config_multiline_2d()
    tx_x = g.tx_origin[:, 0].astype(np.float64)
    xs = np.array([tx_x[0] - 1e-3, tx_x[10] + 1e-5, 0.5 * (tx_x[20] + tx_x[21]) - 1e-6, tx_x[-1] + 2e-3])
    a = L.aux_geometry(g, xs)
    assert a.line_tx.tolist() == [0, 10, 20, 63]
    np.testing.assert_allclose(a.line_origin[:, 0], xs.astype(np.float32))
    assert np.all(a.line_dir == np.float32([0, 0, 1])) and a.n_lines == 4
    assert a.n_depth == g.n_depth and a.tx_origin is g.tx_origin


def test_cnr_regions_are_three_quarters_and_the_ring():
    """Inside 0.75 R against 1.25 R .. 1.75 R: a cyst whose edge zone (0.75 R .. 1.25 R) holds
    outliers does not change the measure."""
    lx = np.linspace(-10e-3, 10e-3, 401)
    z = np.linspace(0, 40e-3, 801)
    X, Z = np.meshgrid(lx, z, indexing="ij")
    d2 = X ** 2 + (Z - 20e-3) ** 2
    R = 4e-3
    inside = d2 <= (0.75 * R) ** 2
    ring_m = (d2 >= (1.25 * R) ** 2) & (d2 <= (1.75 * R) ** 2)
    env = np.where(inside, 0.0, 1.0) + np.where(ring_m, (X > 0) * 1.0, 0.0)
    env = np.where(~inside & (d2 < (1.25 * R) ** 2), 100.0, env)
    c = L.cnr(env, lx, z, [(0.0, 20e-3, R)])
    ring = env[ring_m]
    exact = abs(0.0 - ring.mean()) / np.sqrt(0.0 + ring.var())
    assert abs(c[0] - exact) < 1e-12
