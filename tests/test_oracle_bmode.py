"""Pins of the oracle's envelope detection, log compression and scan conversion
(Sec. 1 pipeline list; Sec. 2 method list items 3-5; the PSF study's Hilbert envelope and
50 dB display range in Sec. 3.2)."""
import numpy as np
import pytest
import scipy.signal

import oracle
import synth
from synth.geometry import ScanGrid


# ------------------------------------------------------------------ envelope

@pytest.mark.parametrize("n", [1024, 2048, 1000, 7])
def test_envelope_of_a_sinusoid_is_its_amplitude(n):
    """Whole-period cosine at a bin strictly between DC and Nyquist: the envelope is flat."""
    k = max(1, n // 5)
    A, ph = 3.7, 0.4
    x = A * np.cos(2 * np.pi * k * np.arange(n) / n + ph)
    np.testing.assert_allclose(oracle.envelope(x), A, rtol=0, atol=1e-12 * A * n)


@pytest.mark.parametrize("n", [1024, 2048, 1000, 33])
def test_envelope_matches_scipy_hilbert(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((3, n))
    np.testing.assert_allclose(oracle.envelope(x), np.abs(scipy.signal.hilbert(x, axis=-1)),
                               rtol=0, atol=1e-12)


def test_envelope_energy_identity():
    """Analytic-signal energy = 2 * signal energy - (DC and Nyquist terms)."""
    n = 512
    rng = np.random.default_rng(2)
    x = rng.standard_normal(n)
    X = np.fft.fft(x)
    want = 2 * np.sum(x * x) - (abs(X[0]) ** 2 + abs(X[n // 2]) ** 2) / n
    assert np.sum(oracle.envelope(x) ** 2) == pytest.approx(want, rel=1e-12)


# ------------------------------------------------------------------ log compression

def test_log_compression_range_identity():
    DR = 50.0
    ref = 123.0
    floor_lvl = ref * 10 ** (-DR / 20)
    env = np.array([ref, floor_lvl, floor_lvl / 3, 0.0, ref / 10, ref / 100])
    B = oracle.log_compress(env, DR, ref=ref)
    np.testing.assert_allclose(B, [1.0, 0.0, 0.0, 0.0, 1 - 20 / DR, 1 - 40 / DR], atol=1e-14)
    rng = np.random.default_rng(0)
    x, y = rng.uniform(floor_lvl * 1.01, ref, 2)
    Bx, By = oracle.log_compress(np.array([x, y]), DR, ref=ref)
    assert Bx - By == pytest.approx(20 * np.log10(x / y) / DR, abs=1e-14)


def test_log_compression_is_scale_free_with_frame_max():
    rng = np.random.default_rng(4)
    env = rng.rayleigh(1.0, 5000)
    np.testing.assert_allclose(oracle.log_compress(env), oracle.log_compress(7.5 * env), atol=1e-14)
    assert oracle.log_compress(env).max() == 1.0


# ------------------------------------------------------------------ scan conversion

def _grid_on_nodes(n_u=8, n_d=20):
    lx = (np.arange(n_u) - 3.5).astype(np.float32) * np.float32(0.5e-3)
    r0, dr = 0.0, float(np.float32(0.25e-3))
    return synth.geometry.scan_grid_2d(lx, r0, dr, n_d, nx=n_u, nz=n_d), lx


def test_scan_2d_identity_on_nodes():
    """Output pixels placed on the line/sample nodes reproduce the input exactly."""
    s, lx = _grid_on_nodes()
    lines = np.random.default_rng(1).standard_normal((s.n_u, s.n_depth))
    iu, jd, ok, U, q = oracle.scan_index_2d(s)
    assert ok.all()
    out = oracle.scan_convert_2d(lines, s)
    np.testing.assert_allclose(out, lines.T, rtol=0, atol=1e-6 * np.abs(lines).max())


def test_scan_2d_reproduces_bilinear_fields_and_fills_outside():
    lx = np.linspace(-5e-3, 5e-3, 17).astype(np.float32)
    n_d = 64
    s = synth.geometry.scan_grid_2d(lx, 1e-3, 0.5e-3, n_d, nx=41, nz=37)
    s.x0 = float(np.float32(-6e-3))        # widen the grid so some pixels fall outside
    s.hx = float(np.float32(12e-3 / 40))
    s.fill = -7.0
    r = s.r0 + s.dr * np.arange(n_d)
    a, b, c, d = 0.3, 2.0e2, -1.5e2, 4.0e4
    lines = a + b * lx.astype(np.float64)[:, None] + c * r[None, :] + d * lx.astype(np.float64)[:, None] * r[None, :]
    out = oracle.scan_convert_2d(lines, s)
    iu, jd, ok, U, q = oracle.scan_index_2d(s)
    X = s.x0 + np.arange(s.nx) * s.hx
    Z = s.z0 + np.arange(s.nz) * s.hz
    XX, ZZ = np.meshgrid(X, Z)
    want = a + b * XX + c * ZZ + d * XX * ZZ
    assert (~ok).any() and ok.any()
    np.testing.assert_allclose(out[ok], want[ok], rtol=0, atol=1e-6)
    assert np.all(out[~ok] == -7.0)
    assert np.all(np.abs(X[(~ok).any(0)]) > 5e-3 - 1e-9)


def test_scan_3d_reproduces_trilinear_fields():
    g = synth.config_volume_3d()
    s = g.scan
    ut = s.line_u.astype(np.float64)
    r = s.r0 + s.dr * np.arange(s.n_depth)
    U, V, Rr = np.meshgrid(ut, ut, r, indexing="ij")       # [v][u][r]
    f = lambda u, v, rr: 0.5 + 2 * u - 3 * v + 40 * rr + 5 * u * v + 70 * u * rr - 10 * u * v * rr
    lines = f(np.broadcast_to(ut[None, :, None], U.shape), np.broadcast_to(ut[:, None, None], U.shape),
              Rr).reshape(s.n_v * s.n_u, s.n_depth)
    zs = [5, 40, 90, 127]
    out = oracle.scan_convert_3d(lines, s, z_slices=zs)
    iu, iv, jd, ok, Uq, Vq, q = oracle.scan_index_3d(s, z_slices=zs)
    assert ok.sum() > 1000
    want = f(Uq.astype(np.float64), Vq.astype(np.float64), s.r0 + s.dr * q.astype(np.float64))
    np.testing.assert_allclose(out[ok], want[ok], rtol=0, atol=1e-9)
    assert np.all(out[~ok] == s.fill)


def test_scan_3d_inside_is_the_pyramid():
    """A voxel is inside iff its tangents lie within the steering tables and its range within
    the record; the apex slab z <= 0 never is."""
    g = synth.config_volume_3d()
    s = g.scan
    iu, iv, jd, ok, U, V, q = oracle.scan_index_3d(s, z_slices=[0, 64, 127])
    tmax = float(s.line_u[-1])
    x = s.x0 + np.arange(s.nx) * s.hx
    z = s.z0 + np.array([0, 64, 127]) * s.hz
    inside_u = np.abs(x[None, :] / z[:, None]) <= tmax * (1 + 1e-6)
    assert np.all(ok.any(1) <= inside_u)
