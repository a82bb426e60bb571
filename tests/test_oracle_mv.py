"""Pins of the minimum-variance oracle: the distortionless constraint, optimality (KKT),
closed forms for coherent and heavily loaded data, and interference suppression."""
import numpy as np
import pytest

from oracle import mv


def test_constraint_and_full_aperture_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((20, 128))
    wf, y, w = mv.mv_weights(x)
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(wf.sum(1), 1.0, atol=1e-12)
    np.testing.assert_allclose(y, (wf * x).sum(1), atol=1e-12)


def test_kkt_and_optimality():
    """A w = lambda 1 with lambda = 1 / (1^T A^-1 1), and no feasible perturbation lowers w^T A w."""
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 128)) * np.linspace(1, 3, 128)
    A = mv.loaded(mv.covariance(x, 32), 1e-2)
    wf, y, w = mv.mv_weights(x)
    for p in range(5):
        Aw = A[p] @ w[p]
        np.testing.assert_allclose(Aw, Aw.mean(), rtol=1e-10)
        lam = 1.0 / np.linalg.solve(A[p], np.ones(32)).sum()
        assert Aw.mean() == pytest.approx(lam, rel=1e-10)
        base = w[p] @ A[p] @ w[p]
        for _ in range(20):
            d = rng.standard_normal(32)
            d -= d.mean()                       # keeps 1^T (w + d) = 1
            u = w[p] + 1e-2 * d
            assert u @ A[p] @ u >= base


def test_covariance_definition_identities():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 40))
    R = mv.covariance(x, 8)
    np.testing.assert_allclose(R, np.transpose(R, (0, 2, 1)), atol=0)
    K = 40 - 8 + 1
    tr = np.array([sum(np.sum(x[p, l:l + 8] ** 2) for l in range(K)) / K for p in range(3)])
    np.testing.assert_allclose(np.trace(R, axis1=1, axis2=2), tr, rtol=1e-12)
    assert np.all(np.linalg.eigvalsh(R) > -1e-12)


def test_coherent_signal_gives_uniform_weights():
    """Identical samples on every element: R = c^2 1 1^T, whose loaded inverse maps 1 to a
    multiple of 1, so w = 1/L and the output is c."""
    c = 3.5
    x = np.full((2, 128), c)
    wf, y, w = mv.mv_weights(x)
    np.testing.assert_allclose(w, 1.0 / 32, atol=1e-14)
    np.testing.assert_allclose(y, c, rtol=1e-12)


def test_heavy_loading_tends_to_uniform_subaperture_weights():
    """Loading -> infinity: w -> 1/L and w_full -> the triangular-edged average of the K
    overlapping subapertures (count of subapertures containing e) / (K L)."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 128))
    wf, y, w = mv.mv_weights(x, loading=1e9)
    np.testing.assert_allclose(w, 1.0 / 32, atol=1e-9)
    K = 97
    count = np.array([min(e, 31) - max(0, e - K + 1) + 1 for e in range(128)])
    np.testing.assert_allclose(wf, np.broadcast_to(count / (K * 32), wf.shape), atol=1e-9)


def test_interference_is_suppressed():
    """Broadside signal (equal on all elements) plus a 20x stronger interferer with a linear
    phase ramp across the aperture: MV keeps the signal (distortionless) and nulls the
    interferer, which uniform subaperture weights let through."""
    M, L = 128, 32
    e = np.arange(M)
    rng = np.random.default_rng(4)
    n = 64
    s = rng.standard_normal(n)
    phase = rng.uniform(0, 2 * np.pi, n)
    x = s[:, None] + 20.0 * np.cos(2 * np.pi * 0.11 * e[None, :] + phase[:, None])
    wf, y, w = mv.mv_weights(x, L=L, loading=1e-3)
    y_uniform = (mv.expand(np.full((n, L), 1.0 / L), M) * x).sum(1)
    err_mv, err_uniform = np.median(np.abs(y - s)), np.median(np.abs(y_uniform - s))
    assert err_uniform > 0.02          # the interferer leaks through fixed weights ...
    assert err_mv < 0.05 * err_uniform  # ... and is nulled by the adaptive ones


def test_all_zero_pixel_gets_uniform_weights():
    wf, y, w = mv.mv_weights(np.zeros((2, 128)))
    np.testing.assert_allclose(w, 1.0 / 32, atol=1e-15)
    assert np.all(y == 0)


# ---- temporal averaging

def test_averaging_identical_rows_changes_nothing():
    rng = np.random.default_rng(11)
    x = rng.standard_normal((5, 128))
    wf, y, w = mv.mv_weights(x)
    wf3, y3, w3 = mv.mv_weights_averaged(np.repeat(x[:, None], 5, axis=1))
    np.testing.assert_allclose(wf3, wf, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(y3, y, rtol=1e-10, atol=1e-13)


def test_averaged_covariance_is_the_snapshot_covariance():
    """All (depth, subaperture) snapshots stacked into one matrix X [T K, L]: R = X^T X / (T K)."""
    rng = np.random.default_rng(12)
    T, M, L = 7, 64, 16
    x = rng.standard_normal((3, T, M))
    R = mv.covariance_averaged(x, L)
    K = M - L + 1
    for p in range(3):
        X = np.stack([x[p, t, l:l + L] for t in range(T) for l in range(K)])
        np.testing.assert_allclose(R[p], X.T @ X / (T * K), rtol=1e-12, atol=1e-12)


def test_averaging_over_depth_limits_signal_cancellation():
    """Long subapertures (L = 96, 33 snapshots per depth) with a strong interferer whose phase
    changes from depth to depth: the single-depth estimate cancels part of the wanted signal,
    averaging over 9 depths restores it (error at least halved)."""
    M, L, n = 128, 96, 64
    e = np.arange(M)
    err = {}
    for T in (1, 9):
        rng = np.random.default_rng(7)
        xs, ss = [], []
        for _ in range(n):
            s = rng.standard_normal(T)
            ph = rng.uniform(0, 2 * np.pi, T)
            xs.append(s[:, None] + 20.0 * np.cos(2 * np.pi * 0.11 * e[None, :] + ph[:, None])
                      + 0.1 * rng.standard_normal((T, M)))
            ss.append(s[T // 2])
        _, y, _ = mv.mv_weights_averaged(np.array(xs), L=L, loading=1e-3)
        err[T] = np.median(np.abs(y - np.array(ss)))
    assert err[9] < 0.5 * err[1]


# ---- analytic-signal (complex) covariance

def test_complex_estimator_on_real_data_is_the_real_estimator():
    rng = np.random.default_rng(21)
    x = rng.standard_normal((6, 128)) * np.linspace(1, 2, 128)
    wf, y, w = mv.mv_weights(x)
    wfc, yc, wc = mv.mv_weights_complex(x + 0j)
    np.testing.assert_allclose(wc, w, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(wfc, wf, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(yc, y, rtol=1e-10, atol=1e-12)


def test_complex_weights_ignore_a_common_phase():
    """z -> z e^{i phi}: R is unchanged, so are the weights, and y turns by the same phase."""
    rng = np.random.default_rng(22)
    z = rng.standard_normal((4, 128)) + 1j * rng.standard_normal((4, 128))
    wf, y, w = mv.mv_weights_complex(z)
    ph = np.exp(1j * 0.7)
    wf2, y2, w2 = mv.mv_weights_complex(z * ph)
    np.testing.assert_allclose(w2, w, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(y2, y * ph, rtol=1e-10, atol=1e-12)


def test_complex_coherent_signal_gives_uniform_weights():
    c = 2.0 - 1.5j
    wf, y, w = mv.mv_weights_complex(np.full((2, 128), c))
    np.testing.assert_allclose(w, 1.0 / 32, atol=1e-14)
    np.testing.assert_allclose(y, c, rtol=1e-12)


def test_complex_kkt_hermitian_and_optimality():
    """A w = lambda 1 with lambda real and positive; R Hermitian positive semidefinite; no
    perturbation that keeps 1^T w = 1 lowers w^H A w."""
    rng = np.random.default_rng(23)
    z = (rng.standard_normal((4, 128)) + 1j * rng.standard_normal((4, 128))) * np.linspace(1, 3, 128)
    R = mv.covariance_complex(z, 32)
    np.testing.assert_allclose(R, np.conj(np.transpose(R, (0, 2, 1))), atol=0)
    assert np.all(np.linalg.eigvalsh(R) > -1e-12)
    A = mv.loaded(R, 1e-2)
    wf, y, w = mv.mv_weights_complex(z)
    np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-12)
    for p in range(4):
        Aw = A[p] @ w[p]
        lam = Aw.mean()
        assert abs(lam.imag) < 1e-12 * abs(lam) and lam.real > 0
        np.testing.assert_allclose(Aw, lam, rtol=1e-10)
        base = np.real(np.conj(w[p]) @ A[p] @ w[p])
        for _ in range(20):
            d = rng.standard_normal(32) + 1j * rng.standard_normal(32)
            d -= d.mean()
            u = w[p] + 1e-2 * d
            assert np.real(np.conj(u) @ A[p] @ u) >= base


def test_complex_interference_is_nulled():
    """Broadside complex signal plus a 20x stronger plane-wave interferer with a linear phase
    ramp across the aperture: the signal passes, the interferer is nulled."""
    M, L = 128, 32
    e = np.arange(M)
    rng = np.random.default_rng(24)
    n = 64
    s = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    ph = rng.uniform(0, 2 * np.pi, n)
    z = s[:, None] + 20.0 * np.exp(1j * (2 * np.pi * 0.11 * e[None, :] + ph[:, None]))
    wf, y, w = mv.mv_weights_complex(z, L=L, loading=1e-3)
    y_uniform = (mv.expand(np.full((n, L), 1.0 / L), M) * z).sum(1)
    err_mv, err_uniform = np.median(np.abs(y - s)), np.median(np.abs(y_uniform - s))
    assert err_uniform > 0.02
    assert err_mv < 0.05 * err_uniform


def test_analytic_channels_match_scipy_hilbert():
    import scipy.signal
    rng = np.random.default_rng(25)
    rf = rng.integers(-3000, 3000, size=(2, 3, 4, 250)).astype(np.int16)
    za = mv.analytic_channels(rf)
    np.testing.assert_allclose(za, scipy.signal.hilbert(rf.astype(np.float64), axis=-1), atol=1e-9)
    np.testing.assert_allclose(za.real, rf, atol=1e-9)


def test_complex_gather_real_part_is_the_real_gather():
    """The analytic signal's real part is the channel data itself, so the real part of the
    complex gather equals the (C) delay-gather of the int16 data at the same taps."""
    import oracle
    import synth
    g = synth.config_tiny(n_el=6, n_tx=2, lines_per_tx=3, n_samples=96)
    rng = np.random.default_rng(26)
    rf = rng.integers(-3000, 3000, size=(2, g.n_tx, g.n_el, g.n_samples)).astype(np.int16)
    za = mv.analytic_channels(rf)
    pix = np.stack([rng.integers(0, 2, 40), rng.integers(0, g.n_lines, 40), rng.integers(0, g.n_depth, 40)], 1)
    z = mv.delay_gather_complex(g, za, pix)
    x = oracle.delay_gather(g, rf, pix)
    np.testing.assert_allclose(z.real, x, atol=1e-9)
    assert np.abs(z.imag).max() > 0
