"""Pins of the oracle's transform, magnitude and normalisation steps.

Each check ties the oracle to something other than itself: an independent FP64
FFT library, Parseval's identity, the closed-form spectrum of pure tones, and
the quantisation-error bound of noiseless synthetic frames.
"""

import json
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def _rand_frames(rng, f, n, lim=8192):
    return rng.integers(-lim, lim, size=(f, n)).astype(np.int16)


@pytest.mark.parametrize("n", [8, 16, 512, 1024, 2048, 4096, 8192])
def test_dft_matches_numpy_rfft(n):
    rng = np.random.default_rng(n)
    fr = _rand_frames(rng, 3, n)
    bins = np.arange(n // 2 + 1) if n <= 512 else rng.choice(n // 2 + 1, 200, replace=False)
    re, im = oracle.dft_at_bins(fr, bins)
    ref = np.fft.rfft(fr.astype(np.float64), axis=1)[:, bins]
    scale = np.abs(ref).max()
    assert np.max(np.abs((re + 1j * im) - ref)) <= 1e-12 * scale * np.sqrt(n)


@pytest.mark.parametrize("n", [16, 1024, 4096])
def test_parseval(n):
    rng = np.random.default_rng(1 + n)
    fr = _rand_frames(rng, 1, n)
    x = fr[0].astype(np.float64)
    spec = oracle.full_dft(fr[0])
    p = np.abs(spec) ** 2
    lhs = float(x @ x)
    rhs = (p[0] + 2.0 * p[1:n // 2].sum() + p[n // 2]) / n
    assert abs(lhs - rhs) <= 1e-12 * lhs


@pytest.mark.parametrize("k0", [1, 7, 100, 511])
def test_pure_tone_placement(k0):
    n = 1024
    t = np.arange(n)
    amp = 3000.0
    for phase in (0.0, 0.3, 2.0):
        x = amp * np.cos(2 * np.pi * k0 * t / n + phase)
        # exact integers would quantise; use a frame whose float64 cast is exact by
        # evaluating the transform on the int16-rounded tone and on the float tone bound
        fr = np.rint(x).astype(np.int16)[None, :]
        spec = oracle.full_dft(fr[0])
        mag = np.abs(spec)
        # rounding the tone to integers changes each bin by at most sum|e_t| <= N/2
        assert abs(mag[k0] - amp * n / 2) <= n / 2
        others = np.delete(mag, k0)
        assert others.max() <= n / 2


def test_dc_and_nyquist():
    n = 64
    dc = np.full((1, n), 1234, dtype=np.int16)
    spec = oracle.full_dft(dc[0])
    assert spec[0].real == pytest.approx(1234 * n, rel=1e-15)
    assert np.abs(spec[1:]).max() <= 1e-9 * 1234 * n
    ny = (1000 * (-1) ** np.arange(n)).astype(np.int16)
    spec = oracle.full_dft(ny)
    assert abs(spec[n // 2]) == pytest.approx(1000 * n, rel=1e-15)
    assert np.abs(spec[: n // 2]).max() <= 1e-9 * 1000 * n


def test_linearity_and_int16_extremes():
    rng = np.random.default_rng(5)
    n = 256
    bins = np.arange(1, 100)
    a = _rand_frames(rng, 1, n, 10000)
    b = _rand_frames(rng, 1, n, 10000)
    ra, ia = oracle.dft_at_bins(a, bins)
    rb, ib = oracle.dft_at_bins(b, bins)
    rs, is_ = oracle.dft_at_bins((a.astype(np.int32) + b).astype(np.int16), bins)
    assert np.allclose(rs, ra + rb, atol=1e-8) and np.allclose(is_, ia + ib, atol=1e-8)
    ext = np.where(np.arange(n) % 3 == 0, -32768, 32767).astype(np.int16)[None, :]
    re, im = oracle.dft_at_bins(ext, np.arange(n // 2 + 1))
    ref = np.fft.rfft(ext.astype(np.float64), axis=1)
    assert np.max(np.abs(re + 1j * im - ref)) <= 1e-9 * np.abs(ref).max()
    zero = np.zeros((2, n), dtype=np.int16)
    assert np.all(oracle.tooth_magnitudes(zero, bins) == 0.0)


def test_rejects_non_int16():
    with pytest.raises(TypeError):
        oracle.dft_at_bins(np.zeros((1, 8), dtype=np.int32), [1])


def test_noiseless_teeth_amplitudes_closed_form():
    """A noiseless quantised frame holds tooth amplitudes g A_i N/2 up to the
    quantisation error, whose per-bin standard deviation is sqrt(N/24) in each
    of Re and Im (uniform rounding error of variance 1/12 per sample)."""
    spec = synth.spec_tiny()
    bt = synth.make_batch(spec, 8, seed=3, noise=False)
    m = oracle.tooth_magnitudes(bt.frames, spec.bins)
    i = np.arange(spec.k)
    u = 2.0 * (i[None, :] - bt.centre[:, None]) / bt.width[:, None]
    amp = bt.baseline[:, None] * (1.0 - bt.depth[:, None] / (1.0 + u * u))
    expect = bt.gain * amp * spec.n / 2
    sd = np.sqrt(spec.n / 24.0)
    assert np.max(np.abs(m - expect)) <= 6.0 * sd
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins)
    assert np.max(np.abs(ref - bt.gain * spec.n / 2)) <= 6.0 * sd
    y = oracle.normalize(m, ref)
    assert np.max(np.abs(y - amp)) <= 2e-3


def test_normalize_rejects_bad_reference():
    with pytest.raises(ValueError):
        oracle.normalize(np.ones((2, 3)), np.array([1.0, 0.0, 1.0]))
    with pytest.raises(ValueError):
        oracle.normalize(np.ones((2, 3)), np.array([1.0, np.nan, 1.0]))


def test_paper_geometry_fixture():
    """The tiny workload's geometry follows the paper's printed numbers: beat
    tones at the 51 MHz offset plus multiples of the 10 MHz comb spacing, and a
    cavity linewidth FSR/finesse of about 8 teeth."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_geometry.json")))
    c = g["speed_of_light_m_s"]["value"]
    fsr = c / (2.0 * g["cavity_length_m"]["value"])
    linewidth = fsr / g["cavity_finesse"]["value"]
    teeth = linewidth / g["comb_spacing_hz"]["value"]
    assert 7.9 < teeth < 8.1
    assert synth.spec_tiny().width == (8.0, 8.0)
    bin_hz = 1.024e9 / 1024
    n = np.arange(-55, 45)
    beat = np.abs(g["lo_shift_hz"]["value"] + g["comb_spacing_hz"]["value"] * n)
    assert np.array_equal(synth.tooth_bins_paper_c1(), (beat / bin_hz).astype(np.int32))
    span = 100 * g["comb_spacing_hz"]["value"]
    assert span <= g["comb_span_hz"]["value"]


def test_reference_is_mean_of_amplitudes_over_frames():
    """Three reference frames whose teeth have exact integer samples (DC,
    N/4 and Nyquist) with different amplitudes and phases: the reference is
    the arithmetic mean of the per-frame amplitudes, which differs from their
    sum, their median, their RMS and the amplitude of the complex mean."""
    n = 1024
    t = np.arange(n)
    quarter_cos = np.array([1, 0, -1, 0])[t % 4]
    quarter_sin = np.array([0, 1, 0, -1])[t % 4]        # the same tone, 90 degrees on
    nyq = np.where(t % 2 == 0, 1, -1)
    amps = [(3, 100, 5), (-7, 200, 11), (20, 900, -2)]   # (DC, N/4 tone, Nyquist)
    frames = []
    for j, (a0, a1, a2) in enumerate(amps):
        tone = quarter_cos if j != 1 else quarter_sin
        frames.append(a0 + a1 * tone + a2 * nyq)
    frames = np.array(frames, dtype=np.int16)
    bins = [0, n // 4, n // 2]
    ref = oracle.reference_spectrum(frames, bins)
    per_frame = np.array([[abs(a0) * n, abs(a1) * n / 2, abs(a2) * n] for a0, a1, a2 in amps])
    want = per_frame.mean(axis=0)
    assert np.allclose(ref, want, rtol=1e-12)
    assert not np.allclose(want, np.median(per_frame, axis=0))
    assert not np.allclose(want, np.sqrt((per_frame ** 2).mean(axis=0)))
    coherent = np.abs(np.fft.rfft(frames.astype(np.float64), axis=1).mean(axis=0)[bins])
    assert abs(want[1] - coherent[1]) > 1.0


def test_paper_geometry_2200_int8():
    """The paper's frames: 2200 int8 samples at 2.2 GS/s, teeth |51 + 10 n| MHz
    (n = -115..104) on distinct 1 MHz bins.  The DFT of int8 frames matches
    numpy's FFT, and a noiseless 8-bit comb puts each tooth's amplitude at
    A g N / 2 within the quantisation bound."""
    bins = synth.tooth_bins_paper_2200()
    assert len(bins) == 220 and len(np.unique(bins)) == 220
    assert bins.min() == 1 and bins.max() == 1099
    rng = np.random.default_rng(22)
    fr = rng.integers(-128, 128, size=(3, 2200)).astype(np.int8)
    re, im = oracle.dft_at_bins(fr, bins)
    ref = np.fft.rfft(fr.astype(np.float64), axis=1)[:, bins]
    assert np.max(np.abs((re + 1j * im) - ref)) <= 1e-12 * np.abs(ref).max() * np.sqrt(2200)
    spec = synth.spec_paper8()
    bt = synth.make_batch(spec, 4, seed=3, noise=False)
    assert bt.frames.dtype == np.int8 and bt.frames.shape == (4, 2200)
    m = oracle.tooth_magnitudes(bt.ref_frames, spec.bins)[0]
    # a unit comb scaled by the gain: every tooth at g N / 2 up to the 8-bit
    # rounding, whose error per bin is at most N/2 (|e_t| <= 1/2)
    assert np.max(np.abs(m - bt.gain * 2200 / 2)) <= 2200 / 2
    with pytest.raises(TypeError):
        oracle.frames_to_float(fr.astype(np.int32))
