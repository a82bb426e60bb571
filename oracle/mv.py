"""Minimum-variance (Capon) apodization oracle -- TEST INFRASTRUCTURE ONLY.

Adaptive receive weights computed from the delayed channel samples of one pixel, used as
training targets for the learned apodization.  Not a step the paper describes: its receive
beamformer is delay and sum (Sec. 2 method list item 2); minimum variance is the adaptive
extension in the spirit of the paper's "software defined" pipeline, following the spatially
smoothed, diagonally loaded estimator of Synnevaag, Austeng and Holm (2007):

  x      delayed samples of the M elements (real), subaperture length L, K = M - L + 1
  R      = (1/K) sum_l x_l x_l^T,  x_l = x[l : l+L]                (spatial smoothing)
  A      = R + eps I,  eps = loading * trace(R) / L                   (diagonal loading)
  v      = A^{-1} 1  by Cholesky factorisation A = C C^T (float64)
  w      = v / (1^T v)                                                (distortionless: 1^T w = 1)
  w_full[e] = (1/K) sum_{l : 0 <= e - l < L} w[e - l]                 (weights on the full aperture)
  y      = w_full^T x = (1/K) sum_l w^T x_l

Everything is float64; numpy's Cholesky and triangular solves are the library steps.

Analytic-signal (complex) covariance (the usual form of the same estimator, not in the
paper): the channel data is first turned into its analytic signal, trace by trace (the
length-S DFT method of the Hilbert envelope), the complex traces are delayed with the same
taps as the real ones (binary32 index rule, interpolation at the float64 delay), and
  R      = (1/K) sum_l z_l z_l^H                                       (Hermitian)
  A      = R + eps I,  eps = loading * trace(R) / L
  v      = A^{-1} 1  by the complex Cholesky factorisation A = C C^H
  w      = v / (1^T v)                                                 (w^H 1 = 1)
  y      = (1/K) sum_l w^H z_l = w_full^H z                            (complex; |y| is the envelope)
This is the minimum-variance beamformer of Capon with a unit steering vector after delay;
for real data it reduces to the real estimator above, number for number.

Temporal averaging (a common refinement of the same estimator, not in the paper): the
covariance also averages over T neighbouring depth samples of the pixel's line,
  R = (1/(T K)) sum_tau sum_l x_{tau,l} x_{tau,l}^T,
with x_tau the delayed samples at depth j + tau - (T-1)/2 (T odd); the weights then apply to
the pixel's own samples (tau = (T-1)/2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def covariance(x: np.ndarray, L: int) -> np.ndarray:
    """Spatially smoothed sample covariance, x: [P, M] -> [P, L, L]."""
    x = np.asarray(x, dtype=np.float64)
    P, M = x.shape
    K = M - L + 1
    R = np.zeros((P, L, L))
    for l in range(K):
        xl = x[:, l:l + L]
        R += xl[:, :, None] * xl[:, None, :]
    return R / K


def covariance_averaged(x: np.ndarray, L: int) -> np.ndarray:
    """Spatially and temporally smoothed covariance, x: [P, T, M] -> [P, L, L]: the mean of the
    per-depth smoothed covariances."""
    x = np.asarray(x, dtype=np.float64)
    P, T, M = x.shape
    R = np.zeros((P, L, L))
    for t in range(T):
        R += covariance(x[:, t], L)
    return R / T


def loaded(R: np.ndarray, loading: float) -> np.ndarray:
    """R + eps I with eps = loading * trace(R) / L; all-zero data (trace 0) gets eps = 1,
    which makes the weights uniform."""
    L = R.shape[-1]
    tr = np.real(np.trace(R, axis1=-2, axis2=-1))
    eps = np.where(tr > 0, loading * tr / L, 1.0)
    return R + eps[:, None, None] * np.eye(L)


def solve_ones(A: np.ndarray) -> np.ndarray:
    """v = A^{-1} 1 through the Cholesky factor of each A (float64)."""
    P, L, _ = A.shape
    v = np.empty((P, L))
    ones = np.ones(L)
    for p in range(P):
        C = np.linalg.cholesky(A[p])
        z = scipy.linalg.solve_triangular(C, ones, lower=True)
        v[p] = scipy.linalg.solve_triangular(C.T, z, lower=False)
    return v


def expand(w: np.ndarray, M: int) -> np.ndarray:
    """Subaperture weights [P, L] -> full-aperture weights [P, M]."""
    P, L = w.shape
    K = M - L + 1
    wf = np.zeros((P, M), dtype=np.result_type(w, np.float64))
    for l in range(K):
        wf[:, l:l + L] += w
    return wf / K


def mv_weights(x: np.ndarray, L: int = 32, loading: float = 1e-2):
    """Returns (w_full [P, M], y [P], w [P, L]) for delayed samples x [P, M]."""
    x = np.asarray(x, dtype=np.float64)
    A = loaded(covariance(x, L), loading)
    v = solve_ones(A)
    w = v / v.sum(axis=1, keepdims=True)
    wf = expand(w, x.shape[1])
    y = np.einsum("pm,pm->p", wf, x)
    return wf, y, w


def mv_weights_averaged(x: np.ndarray, L: int = 32, loading: float = 1e-2):
    """Minimum variance with temporal averaging: x [P, T, M] (T odd, the pixel's own samples
    in the middle row) -> (w_full [P, M], y [P], w [P, L])."""
    x = np.asarray(x, dtype=np.float64)
    A = loaded(covariance_averaged(x, L), loading)
    v = solve_ones(A)
    w = v / v.sum(axis=1, keepdims=True)
    wf = expand(w, x.shape[2])
    y = np.einsum("pm,pm->p", wf, x[:, x.shape[1] // 2])
    return wf, y, w


# ---- analytic-signal (complex) covariance

def analytic_channels(rf: np.ndarray) -> np.ndarray:
    """Analytic signal of every channel trace (last axis, circular, length S), complex128."""
    from . import analytic_filter
    x = np.asarray(rf, dtype=np.float64)
    return np.fft.ifft(np.fft.fft(x, axis=-1) * analytic_filter(x.shape[-1]), axis=-1)


def delay_gather_complex(g, za: np.ndarray, pix) -> np.ndarray:
    """Delayed complex samples z [n_pix, n_el] of analytic channel data za [F, n_tx, n_el, S] at
    pixels pix [n][3] (frame, line, depth): the delay-and-sum taps -- valid by the binary32
    index rule, interpolated linearly at the float64 delay (clamped into the record) -- applied
    to the real and imaginary parts alike; 0 where the tap is invalid or the line has no
    transmit."""
    from . import tau64, tof32
    za = np.asarray(za)
    pix = np.asarray(pix, dtype=np.int64).reshape(-1, 3)
    S = za.shape[-1]
    i0, _, _, valid = tof32(g, pix[:, 1:])
    tau = np.clip(tau64(g, pix[:, 1:]), 0.0, S - 1)
    fl = np.floor(tau)
    ph = tau - fl
    i = fl.astype(np.int64)
    i1 = np.minimum(i + 1, S - 1)
    t = np.asarray(g.line_tx)[pix[:, 1]]
    ok_line = (t >= 0) & (t < g.n_tx)
    f = pix[:, 0][:, None]
    tt = np.where(ok_line, t, 0)[:, None]
    e = np.arange(g.n_el)[None, :]
    z = (1.0 - ph) * za[f, tt, e, i] + ph * za[f, tt, e, i1]
    return np.where(valid & ok_line[:, None], z, 0.0)


def covariance_complex(z: np.ndarray, L: int) -> np.ndarray:
    """Spatially smoothed Hermitian covariance, z: [P, M] complex -> [P, L, L]."""
    z = np.asarray(z, dtype=np.complex128)
    P, M = z.shape
    K = M - L + 1
    R = np.zeros((P, L, L), dtype=np.complex128)
    for l in range(K):
        zl = z[:, l:l + L]
        R += zl[:, :, None] * np.conj(zl[:, None, :])
    return R / K


def solve_ones_complex(A: np.ndarray) -> np.ndarray:
    """v = A^{-1} 1 through the Cholesky factor A = C C^H of each Hermitian A."""
    P, L, _ = A.shape
    v = np.empty((P, L), dtype=np.complex128)
    ones = np.ones(L, dtype=np.complex128)
    for p in range(P):
        C = np.linalg.cholesky(A[p])
        u = scipy.linalg.solve_triangular(C, ones, lower=True)
        v[p] = scipy.linalg.solve_triangular(np.conj(C.T), u, lower=False)
    return v


def mv_weights_complex(z: np.ndarray, L: int = 32, loading: float = 1e-2):
    """Minimum variance on complex (analytic) delayed samples z [P, M]:
    returns (w_full [P, M], y [P], w [P, L]), all complex, y = w_full^H z."""
    z = np.asarray(z, dtype=np.complex128)
    A = loaded(covariance_complex(z, L), loading)
    v = solve_ones_complex(A)
    w = v / v.sum(axis=1, keepdims=True)
    wf = expand(w, z.shape[1])
    y = np.einsum("pm,pm->p", np.conj(wf), z)
    return wf, y, w
