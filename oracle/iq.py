"""Envelope by IQ demodulation with frequency compounding -- CPU oracle (test infrastructure).

The paper's own envelope node demodulates each beamformed line to baseband (IQ) and
compounds several frequency bands from a bank of configurable bandpasses (Sec. 2 method list
item 3).  The paper prints no formula; this oracle follows the textbook steps in the paper's
order, in float64:

  1. for every band k (centre frequency f_k): mix the line down, y[t] exp(-2 pi i f_k t / fs);
  2. low-pass the mixed signal with the FIR prototype h (length L odd, centred: output sample n
     uses inputs n - c .. n + c, c = (L - 1) / 2, zeros outside the line);
  3. take the magnitude of the complex baseband signal, times 2 (a tone of amplitude A at f_k
     then has envelope A);
  4. compound: average the K band envelopes.

The prototype is a Hamming-windowed sinc with cutoff B / 2 (B the band width), normalised to
unit gain at DC.

Parity of the GPU kernel is against `envelope_iq` below; `envelope_iq_mixing` evaluates the
same definition literally (mix, filter, magnitude) and pins the algebra of the fast form.
"""
from __future__ import annotations

import numpy as np


def lowpass_taps(n_taps: int, bandwidth: float, fs: float) -> np.ndarray:
    """Hamming-windowed sinc low-pass, cutoff bandwidth / 2, unit DC gain, float64 [n_taps]."""
    assert n_taps % 2 == 1 and n_taps >= 3
    c = (n_taps - 1) // 2
    m = np.arange(n_taps) - c
    fc = 0.5 * bandwidth / fs                     # cycles per sample
    h = 2.0 * fc * np.sinc(2.0 * fc * m)
    w = 0.54 - 0.46 * np.cos(2.0 * np.pi * np.arange(n_taps) / (n_taps - 1))
    h = h * w
    return h / h.sum()


def band_taps(n_taps: int, bandwidth: float, fs: float, freqs) -> np.ndarray:
    """Complex bandpass taps g_k[m] = h[m] exp(2 pi i f_k (m - c) / fs), complex128 [K][L]:
    |sum_m g_k[m] y[n + c - m]| equals the magnitude of the mixed-then-filtered signal."""
    h = lowpass_taps(n_taps, bandwidth, fs)
    c = (n_taps - 1) // 2
    m = np.arange(n_taps) - c
    f = np.asarray(freqs, np.float64)[:, None]
    return h[None, :] * np.exp(2j * np.pi * f * m[None, :] / fs)


def envelope_iq(y, fs: float, freqs, bandwidth: float, n_taps: int) -> np.ndarray:
    """Compounded IQ envelope of rows y [..., N] (float64 result, same shape)."""
    y = np.asarray(y, np.float64)
    g = band_taps(n_taps, bandwidth, fs, freqs)
    c = (n_taps - 1) // 2
    n = y.shape[-1]
    yp = np.zeros(y.shape[:-1] + (n + 2 * c,))
    yp[..., c:c + n] = y
    out = np.zeros(y.shape, np.float64)
    for gk in g:
        z = np.zeros(y.shape, np.complex128)
        for mm in range(n_taps):
            # y[n + c - m] sits at padded index n + 2c - m
            z += gk[mm] * yp[..., 2 * c - mm:2 * c - mm + n]
        out += 2.0 * np.abs(z)
    return out / len(g)


def envelope_iq_mixing(y, fs: float, freqs, bandwidth: float, n_taps: int) -> np.ndarray:
    """The same envelope evaluated step by step (mix to baseband, low-pass, magnitude,
    average), with explicit loops: for small inputs only."""
    y = np.asarray(y, np.float64)
    h = lowpass_taps(n_taps, bandwidth, fs)
    c = (n_taps - 1) // 2
    n = y.shape[-1]
    t = np.arange(n)
    out = np.zeros(y.shape, np.float64)
    for f in freqs:
        mixed = y * np.exp(-2j * np.pi * f * t / fs)
        base = np.zeros(y.shape, np.complex128)
        for i in range(n):
            for mm in range(n_taps):
                src = i + c - mm
                if 0 <= src < n:
                    base[..., i] += h[mm] * mixed[..., src]
        out += 2.0 * np.abs(base)
    return out / len(freqs)
