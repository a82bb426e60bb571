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
    tr = np.trace(R, axis1=-2, axis2=-1)
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
    wf = np.zeros((P, M))
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
