"""Seeded channel-data (RF) simulator (input generation only).

Forward model: every scatterer k with amplitude a_k echoes a 2-cycle
Gaussian-windowed pulse g(t) = cos(2 pi f0 t) exp(-t^2 / 2 s^2) (envelope FWHM of two
periods, cut at |t| <= 3 s) that reaches element e of transmit t after the focused-wave
travel time: the wave converges on a virtual source at the focus, so the transmit
time is (F +- |p - focus|)/c (a plane wave, infinite focus: (p - o).u / c), plus the
receive path |e - p|/c.  White Gaussian noise at
a stated SNR is added and the frame is quantised to int16 (peak 30000).

Implementation: arrivals are deposited on a grid 16x finer than the sampling grid
(linear split between neighbouring fine bins, accumulated in int64 fixed point so the
result does not depend on summation order), the fine traces are convolved with the
pulse by FFT, and every 16th fine sample is kept.  Runs with torch on the CPU or on a
GPU; the bytes it returns are what both the oracle and the library consume.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .geometry import Geometry

UPSAMPLE = 16
FIX_SCALE = float(2 ** 30)


def pulse_sigma(f0: float) -> float:
    """Gaussian sigma whose envelope FWHM equals two periods of f0."""
    return 2.0 / (f0 * 2.0 * math.sqrt(2.0 * math.log(2.0)))


def pulse(t: torch.Tensor, f0: float) -> torch.Tensor:
    s = pulse_sigma(f0)
    g = torch.cos(2 * math.pi * f0 * t) * torch.exp(-t * t / (2 * s * s))
    return torch.where(t.abs() <= 3 * s, g, torch.zeros_like(g))


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def arrival_samples(g: Geometry, tx: int, pos: torch.Tensor, el: torch.Tensor) -> torch.Tensor:
    """Arrival time, in samples, of each scatterer at each element for transmit `tx`: [n_el, K]."""
    dev = pos.device
    o = torch.tensor(g.tx_origin[tx], dtype=torch.float64, device=dev)
    d = torch.tensor(_unit(g.tx_dir[tx]), dtype=torch.float64, device=dev)
    F = float(g.tx_focus[tx])
    axial = (pos - o) @ d
    if np.isinf(F):
        # plane wave: the wavefront passes the transmit origin at t = 0
        t_tx = axial / g.c
    else:
        focus = o + F * d
        to_focus = torch.linalg.norm(pos - focus, dim=1)
        t_tx = torch.where(axial >= F, F + to_focus, F - to_focus) / g.c
    t_rx = torch.cdist(el, pos) / g.c          # [n_el, K]
    return (t_tx[None, :] + t_rx - g.t0) * g.fs


def simulate_clean(g: Geometry, pos: np.ndarray, amp: np.ndarray, device="cpu",
                   tx_range=None) -> torch.Tensor:
    """Noise-free float64 channel data [n_tx, n_el, S]."""
    dev = torch.device(device)
    S, U = g.n_samples, UPSAMPLE
    n_fine = S * U
    s = pulse_sigma(g.f0)
    half = int(math.ceil(3 * s * g.fs * U)) + 1
    kt = torch.arange(-half, half + 1, dtype=torch.float64, device=dev) / (g.fs * U)
    ker = pulse(kt, g.f0)                                   # fine-grid pulse
    n_fft = 1 << int(math.ceil(math.log2(n_fine + 4 * half + 3)))
    ker_pad = torch.zeros(n_fft, dtype=torch.float64, device=dev)
    ker_pad[: ker.numel()] = ker
    K_f = torch.fft.rfft(ker_pad)
    P = torch.tensor(pos, dtype=torch.float64, device=dev)
    A = torch.tensor(amp, dtype=torch.float64, device=dev)
    E = torch.tensor(g.el_pos.astype(np.float64), device=dev)
    txs = range(g.n_tx) if tx_range is None else tx_range
    out = torch.zeros((len(txs), g.n_el, S), dtype=torch.float64, device=dev)
    off = half            # fine index of arrival u lands at padded position u + half
    L = n_fine + 2 * half + 2
    row = torch.arange(g.n_el, device=dev)[:, None] * L
    for ti, t in enumerate(txs):
        u = arrival_samples(g, t, P, E) * U + off           # [n_el, K] fine position
        i = torch.floor(u)
        fr = u - i
        i = i.long()
        ok = (i >= 0) & (i + 1 < L)
        w0 = torch.round(A[None, :] * (1 - fr) * FIX_SCALE).long()
        w1 = torch.round(A[None, :] * fr * FIX_SCALE).long()
        idx = (row + i)[ok]
        acc = torch.zeros(g.n_el * L, dtype=torch.int64, device=dev)
        acc.index_add_(0, idx, w0[ok])
        acc.index_add_(0, idx + 1, w1[ok])
        fine = acc.view(g.n_el, L).to(torch.float64) / FIX_SCALE
        spec = torch.fft.rfft(fine, n=n_fft, dim=1) * K_f[None, :]
        conv = torch.fft.irfft(spec, n=n_fft, dim=1)
        # arrival at fine index (u - off) convolved with ker centred at +half -> peak at u - off + 2*half
        start = 2 * half
        out[ti] = conv[:, start: start + n_fine: U]
    return out


def band_limited_speckle(g: Geometry, n_tx: int, rms: float, seed: int, device="cpu") -> torch.Tensor:
    """Gaussian noise shaped by the pulse spectrum: a stand-in for fully developed speckle
    when the scatterer count makes a physical simulation too costly."""
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    S = g.n_samples
    s = pulse_sigma(g.f0)
    half = int(math.ceil(3 * s * g.fs)) + 1
    kt = torch.arange(-half, half + 1, dtype=torch.float32, device=dev) / g.fs
    ker = pulse(kt, g.f0)
    ker = ker / torch.linalg.norm(ker)
    out = torch.empty((n_tx, g.n_el, S), dtype=torch.float32, device=dev)
    for t in range(n_tx):
        w = torch.randn((g.n_el, 1, S + 2 * half), generator=gen, device=dev, dtype=torch.float32)
        out[t] = torch.nn.functional.conv1d(w, ker.view(1, 1, -1))[:, 0, :S] * rms
    return out


def add_noise_and_quantize(clean: torch.Tensor, snr_db: float, seed: int, peak: float = 30000.0):
    dev = clean.device
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    rms = torch.sqrt(torch.mean(clean.double() ** 2)).item()
    sigma = rms * 10 ** (-snr_db / 20.0)
    noisy = clean + sigma * torch.randn(clean.shape, generator=gen, device=dev, dtype=clean.dtype)
    m = noisy.abs().max().item()
    scale = peak / m if m > 0 else 1.0
    q = torch.clamp(torch.round(noisy * scale), -32768, 32767).to(torch.int16)
    return q


def simulate_frame(g: Geometry, pos, amp, seed: int, snr_db: float = 40.0, device="cpu",
                   noise: bool = True) -> torch.Tensor:
    """One int16 frame [n_tx, n_el, S]."""
    clean = simulate_clean(g, pos, amp, device=device)
    if not noise:
        m = clean.abs().max().item()
        scale = 30000.0 / m if m > 0 else 1.0
        return torch.clamp(torch.round(clean * scale), -32768, 32767).to(torch.int16)
    return add_noise_and_quantize(clean, snr_db, seed + 7919)


def simulate_volume(g: Geometry, seed: int, snr_db: float = 40.0, device="cpu",
                    speckle_rms: float | None = None, point_amp: float = 10.0) -> torch.Tensor:
    """3D volume: physically simulated point targets plus band-limited speckle stand-in."""
    from .phantom import points_3d
    pp, pa, _ = points_3d(g, amplitude=point_amp)
    clean = simulate_clean(g, pp, pa, device=device).to(torch.float32)
    if speckle_rms is None:
        # expected RMS of 200k unit-variance scatterers spread over the record
        s = pulse_sigma(g.f0)
        tt = torch.arange(-int(3 * s * g.fs) - 1, int(3 * s * g.fs) + 2, dtype=torch.float64) / g.fs
        e_p = float((pulse(tt, g.f0) ** 2).sum())
        speckle_rms = math.sqrt(200_000 * e_p / g.n_samples)
    clean += band_limited_speckle(g, g.n_tx, speckle_rms, seed, device=device)
    return add_noise_and_quantize(clean, snr_db, seed + 7919)
