"""The IQ-demodulation envelope oracle against textbook routines and closed forms (envelope
detection by IQ demodulation with frequency compounding, Sec. 2 method list item 3)."""
import numpy as np
import scipy.signal

from oracle import iq

FS = 40e6


def test_lowpass_prototype_is_the_textbook_hamming_fir():
    for n_taps, bw in [(31, 2e6), (63, 3e6), (15, 8e6)]:
        h = iq.lowpass_taps(n_taps, bw, FS)
        ref = scipy.signal.firwin(n_taps, bw / 2, window="hamming", fs=FS)
        assert np.allclose(h, ref, atol=1e-14)
        assert abs(h.sum() - 1.0) < 1e-14
        assert np.allclose(h, h[::-1])


def test_filter_form_equals_mixing_form():
    rng = np.random.default_rng(0)
    y = rng.standard_normal((3, 40))
    freqs = [4e6, 6.5e6]
    a = iq.envelope_iq(y, FS, freqs, 2.5e6, 15)
    b = iq.envelope_iq_mixing(y, FS, freqs, 2.5e6, 15)
    assert np.abs(a - b).max() < 1e-12


def test_tone_in_band_has_its_amplitude_as_envelope():
    n = np.arange(2048)
    for f, amp, phase in [(5e6, 3.0, 0.3), (4e6, 0.5, 2.0)]:
        y = amp * np.cos(2 * np.pi * f * n / FS + phase)
        env = iq.envelope_iq(y, FS, [f], 2e6, 63)
        inner = env[64:-64]
        assert np.abs(inner - amp).max() <= 5e-3 * amp


def test_tone_outside_the_band_is_rejected():
    n = np.arange(2048)
    y = np.cos(2 * np.pi * 12e6 * n / FS)
    env = iq.envelope_iq(y, FS, [5e6], 2e6, 63)
    assert env[64:-64].max() < 1e-2


def test_compounding_is_the_mean_of_the_bands():
    rng = np.random.default_rng(1)
    y = rng.standard_normal((2, 300))
    freqs = [3.5e6, 5e6, 6.5e6]
    env = iq.envelope_iq(y, FS, freqs, 2e6, 31)
    single = [iq.envelope_iq(y, FS, [f], 2e6, 31) for f in freqs]
    assert np.abs(env - np.mean(single, axis=0)).max() < 1e-12


def test_zero_and_scaling():
    rng = np.random.default_rng(2)
    y = rng.standard_normal(200)
    assert np.all(iq.envelope_iq(np.zeros(200), FS, [5e6], 2e6, 31) == 0.0)
    e1 = iq.envelope_iq(y, FS, [5e6, 6e6], 2e6, 31)
    e2 = iq.envelope_iq(-2.5 * y, FS, [5e6, 6e6], 2e6, 31)
    assert np.abs(e2 - 2.5 * e1).max() < 1e-12
