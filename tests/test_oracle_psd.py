"""Pins of the oracle's displacement PSD (Welch) and mechanical resonance fit
against things other than the oracle: scipy's Welch estimator, Parseval for
a pure tone, the white-noise level, the closed-form spectrum of the
second-order recursion the generator integrates, scipy's MINPACK
Levenberg-Marquardt on the log residuals, and exact recovery of noiseless
model spectra."""

import numpy as np
import pytest
from scipy import signal
from scipy.optimize import least_squares

import synth
from oracle import psd


@pytest.mark.parametrize("seg", [4096, 65536])
def test_welch_matches_scipy(seg):
    rng = np.random.default_rng(seg)
    x = rng.standard_normal(3 * seg + 123) + np.sin(2 * np.pi * 0.0137 * np.arange(3 * seg + 123))
    fs = 1.0e6
    f, p = signal.welch(x, fs=fs, window="hann", nperseg=seg, noverlap=seg // 2,
                        detrend="constant", scaling="density")
    k_lo, nb = seg // 64, seg // 8
    mine = psd.welch_band(x, fs, seg, k_lo, nb)
    assert np.allclose(mine, p[k_lo:k_lo + nb], rtol=1e-10, atol=0)
    # the edges: DC and Nyquist halved like scipy's
    both = psd.welch_band(x, fs, seg, 0, 2)
    assert np.allclose(both, p[:2], rtol=1e-10)
    assert np.allclose(psd.welch_band(x, fs, seg, seg // 2, 1), p[seg // 2], rtol=1e-10)


def test_pure_tone_power_and_white_level():
    seg, fs = 4096, 1.0e6
    t = np.arange(8 * seg)
    a, k0 = 3.0, 300
    x = a * np.cos(2 * np.pi * k0 * t / seg + 0.4)
    p = psd.welch_band(x, fs, seg, 1, seg // 2 - 1)
    assert abs(p.sum() * fs / seg - a * a / 2) < 1e-9      # Parseval, Hann, on-bin tone
    sigma = 0.7
    wn = sigma * np.random.default_rng(1).standard_normal(400 * seg)
    lvl = psd.welch_band(wn, fs, seg, 10, seg // 2 - 20).mean()
    assert abs(lvl / (2 * sigma ** 2 / fs) - 1) < 0.01


def test_resonance_spectrum_matches_the_recursion_closed_form():
    fs, f0, q = 1.0e6, 23.7e3, 115.0
    x = synth.make_displacement(1 << 21, fs, f0, q, drive=1e-3, floor=0.0, drift=0.0, seed=2)
    seg = 1 << 16
    k_lo, nb = int(18e3 * seg / fs), int(12e3 * seg / fs)
    p = psd.welch_band(x, fs, seg, k_lo, nb)
    f = (k_lo + np.arange(nb)) * fs / seg
    r = np.exp(-np.pi * f0 / (q * fs))
    th = 2 * np.pi * f0 * np.sqrt(1 - 1 / (4 * q * q)) / fs
    z = np.exp(-2j * np.pi * f / fs)
    true = 2 * 1e-6 / fs / np.abs(1 - 2 * r * np.cos(th) * z + r * r * z * z) ** 2
    ratio = p / true
    assert abs(np.median(ratio) - 1) < 0.05


def test_oscillator_fit_exact_on_noiseless_model():
    f = np.linspace(15e3, 35e3, 1300)
    truth = np.array([np.log(3e5), 23.7e3, 115.0, np.log(2e-9)])
    s = psd.oscillator(f, truth)
    for p0 in (None, truth * np.array([1.0, 1.003, 0.8, 1.0]) + np.array([0.5, 0, 0, -0.3])):
        p, it, st, chi2 = psd.oscillator_fit(f, s, p0=p0)
        assert st == 0
        assert np.allclose(p, truth, rtol=1e-7, atol=1e-7), (p, truth)


def test_oscillator_fit_agrees_with_minpack_on_noisy_spectrum():
    f = np.linspace(15e3, 35e3, 1300)
    truth = np.array([np.log(3e5), 23.7e3, 115.0, np.log(2e-9)])
    noisy = psd.oscillator(f, truth) * np.exp(0.05 * np.random.default_rng(3).standard_normal(f.size))
    p, it, st, chi2 = psd.oscillator_fit(f, noisy, max_iter=400, tol=1e-15)
    res = least_squares(lambda q: np.log(noisy) - np.log(psd.oscillator(f, q)),
                        psd.start_point(f, noisy), method="lm", xtol=1e-15, ftol=1e-15,
                        gtol=1e-15, max_nfev=100000)
    assert np.allclose(p, res.x, rtol=1e-7, atol=1e-9), (p, res.x)
    assert abs(p[1] - truth[1]) < 0.01 * truth[1] / truth[2]


def test_fit_recovers_the_generator_resonance():
    fs, f0, q = 1.0e6, 23.7e3, 115.0
    x = synth.make_displacement(1 << 22, fs, f0, q, drive=1e-3, floor=2e-3, drift=1e-6, seed=4)
    seg = 1 << 16
    k_lo, nb = int(15e3 * seg / fs), int(20e3 * seg / fs)
    p = psd.welch_band(x, fs, seg, k_lo, nb)
    f = (k_lo + np.arange(nb)) * fs / seg
    fit, it, st, _ = psd.oscillator_fit(f, p)
    assert st == 0
    assert abs(fit[1] / f0 - 1) < 1e-3
    assert abs(fit[2] / q - 1) < 0.1


def test_start_point_rules():
    f = np.arange(100.0)
    p = np.full(100, 2.0)
    p[40:49] = [3, 4, 6, 8, 10, 8, 6, 4, 3]
    sp = psd.start_point(f, p)
    assert sp[1] == 44.0 and np.isclose(np.exp(sp[3]), 2.0)
    # half of the peak's excess (8) over the floor: level 6, reached at 42 and 46
    assert np.isclose(sp[2], 44.0 / 4.0)
    assert np.isclose(np.exp(sp[0]), 8.0 * 44.0 ** 4 / sp[2] ** 2)
