"""Learned adaptive apodization oracle -- TEST INFRASTRUCTURE ONLY.

A small 1D convolutional network maps the delayed channel samples of one pixel to one weight
per element; it is trained to reproduce minimum-variance weights (oracle.mv), and the pixel
value is then sum_e w_e x_e.  Not in the paper (whose beamformer is fixed delay and sum,
Sec. 2 method list item 2); the network shape -- four layers, 32 channels, kernel 5 -- is
the workload's.

  xh   = x / sqrt(mean(x^2) + 1e-12)                     per pixel, over the M elements
  h1   = relu(conv(xh; W1 [32][1][5], b1))               'same' zero padding, cross-correlation
  h2   = relu(conv(h1; W2 [32][32][5], b2))
  h3   = relu(conv(h2; W3 [32][32][5], b3))
  w    = conv(h3; W4 [1][32][5], b4)                     linear output, one weight per element
  loss = mean over pixels and elements of (M w - M w_target)^2

Precision of the GPU kernels, reproduced here: every operand of a product (layer inputs,
weights, and in the backward pass the incoming gradients) is rounded to bfloat16 (round to
nearest even); sums are exact (float64 here, binary32 on the GPU).  Adam keeps float32 master
weights.  Set bf16=False for the exact-arithmetic network (gradient checks).
"""
from __future__ import annotations

import numpy as np

C = 32      # channels
KS = 5      # kernel size
PAD = 2


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def init_params(seed: int = 0):
    """He-style uniform initialisation (float32 master copy)."""
    rng = np.random.default_rng(seed)

    def u(shape, fan_in):
        b = np.sqrt(6.0 / fan_in)
        return rng.uniform(-b, b, shape).astype(np.float32)

    return {
        "W1": u((C, 1, KS), KS), "b1": np.zeros(C, np.float32),
        "W2": u((C, C, KS), C * KS), "b2": np.zeros(C, np.float32),
        "W3": u((C, C, KS), C * KS), "b3": np.zeros(C, np.float32),
        "W4": (u((1, C, KS), C * KS) * 0.1).astype(np.float32), "b4": np.full(1, 0.0, np.float32),
    }


def _shifted(h: np.ndarray) -> np.ndarray:
    """[P, Cin, M] -> [P, Cin, KS, M] with tap t reading position m + t - PAD (zeros outside)."""
    P, Ci, M = h.shape
    hp = np.zeros((P, Ci, M + 2 * PAD))
    hp[:, :, PAD:PAD + M] = h
    return np.stack([hp[:, :, t:t + M] for t in range(KS)], axis=2)


def conv(h: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[p, co, m] = b[co] + sum_{ci, t} W[co, ci, t] h[p, ci, m + t - PAD]."""
    return np.einsum("oct,pctm->pom", W, _shifted(h)) + b[None, :, None]


def normalise(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    return x / np.sqrt(np.mean(x * x, axis=1, keepdims=True) + 1e-12)


def _jittered(v: np.ndarray, jitter, n_terms: int) -> np.ndarray:
    """v with every entry scaled by (1 + u * 2^-24 * sqrt(n_terms)), u uniform in [-1, 1]: the
    size of the rounding error a binary32 accumulator adds to a sum of n_terms products in some
    order.  Used only to measure how often that error moves a bfloat16 rounding (jitter = a
    numpy Generator); None leaves v unchanged."""
    if jitter is None:
        return v
    return v * (1.0 + jitter.uniform(-1.0, 1.0, v.shape) * 2.0 ** -24 * np.sqrt(n_terms))


def forward(params, x: np.ndarray, bf: bool = True, jitter=None):
    """Returns (w [P, M], cache).  x: delayed samples [P, M].  jitter: see _jittered."""
    q = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    W = {k: q(v) for k, v in params.items() if k.startswith("W")}
    b = {k: np.asarray(v, np.float64) for k, v in params.items() if k.startswith("b")}
    a0 = q(_jittered(normalise(x), jitter, x.shape[1]))[:, None, :]
    z1 = _jittered(conv(a0, W["W1"], b["b1"]), jitter, KS)
    a1 = q(np.maximum(z1, 0.0))
    z2 = _jittered(conv(a1, W["W2"], b["b2"]), jitter, C * KS)
    a2 = q(np.maximum(z2, 0.0))
    z3 = _jittered(conv(a2, W["W3"], b["b3"]), jitter, C * KS)
    a3 = q(np.maximum(z3, 0.0))
    w = _jittered(conv(a3, W["W4"], b["b4"])[:, 0, :], jitter, C * KS)
    cache = dict(W=W, a0=a0, z1=z1, a1=a1, z2=z2, a2=a2, z3=z3, a3=a3, bf=bf, jitter=jitter)
    return w, cache


def loss_fn(w: np.ndarray, target: np.ndarray) -> float:
    M = w.shape[1]
    return float(np.mean((M * w - M * np.asarray(target, np.float64)) ** 2))


def _conv_backward(g: np.ndarray, a_in: np.ndarray, W: np.ndarray):
    """Given g = dL/d(out) [P, Co, M] of out = conv(a_in; W, b):
    returns (dW [Co, Ci, KS], db [Co], da_in [P, Ci, M])."""
    sh = _shifted(a_in)                                    # [P, Ci, KS, M]
    dW = np.einsum("pom,pctm->oct", g, sh)
    db = g.sum(axis=(0, 2))
    P, Co, M = g.shape
    gp = np.zeros((P, Co, M + 2 * PAD))
    gp[:, :, PAD:PAD + M] = g
    # da[p, ci, m] = sum_{co, t} W[co, ci, t] g[p, co, m - t + PAD]
    da = np.zeros((P, W.shape[1], M))
    for t in range(KS):
        da += np.einsum("oc,pom->pcm", W[:, :, t], gp[:, :, 2 * PAD - t:2 * PAD - t + M])
    return dW, db, da


def backward(params, cache, w: np.ndarray, target: np.ndarray):
    """Gradients of loss_fn(w, target) with respect to every parameter."""
    q = bf16 if cache["bf"] else (lambda a: np.asarray(a, dtype=np.float64))
    P, M = w.shape
    W = cache["W"]
    g = (2.0 * M * M / (P * M)) * (w - np.asarray(target, np.float64))
    jit = cache.get("jitter")
    g4 = q(_jittered(g, jit, 1))[:, None, :]
    dW4, db4, da3 = _conv_backward(g4, cache["a3"], W["W4"])
    g3 = q(_jittered(da3, jit, KS) * (cache["z3"] > 0))
    dW3, db3, da2 = _conv_backward(g3, cache["a2"], W["W3"])
    g2 = q(_jittered(da2, jit, C * KS) * (cache["z2"] > 0))
    dW2, db2, da1 = _conv_backward(g2, cache["a1"], W["W2"])
    g1 = q(_jittered(da1, jit, C * KS) * (cache["z1"] > 0))
    dW1, db1, _ = _conv_backward(g1, cache["a0"], W["W1"])
    return {"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "W3": dW3, "b3": db3, "W4": dW4, "b4": db4}


class Adam:
    """Adam (Kingma and Ba 2015) on float32 master weights."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(v, dtype=np.float64) for k, v in params.items()}
        self.v = {k: np.zeros_like(v, dtype=np.float64) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = {}
        for k in params:
            g = np.asarray(grads[k], np.float64)
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g * g
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            out[k] = (params[k].astype(np.float64) - self.lr * mh / (np.sqrt(vh) + self.eps)).astype(np.float32)
        return out


def apply_weights(w: np.ndarray, x: np.ndarray, fallback: np.ndarray | None = None) -> np.ndarray:
    """y = sum_e w_e x_e per pixel; pixels with a non-finite weight take `fallback` (DAS)."""
    y = np.sum(np.asarray(w, np.float64) * np.asarray(x, np.float64), axis=1)
    if fallback is not None:
        bad = ~np.all(np.isfinite(w), axis=1)
        y[bad] = np.asarray(fallback, np.float64)[bad]
    return y
