"""Seeded generator of digitised comb-tooth heterodyne frames.

Physical picture (paper, Experimental Setup): an electro-optic comb with 10 MHz
tooth spacing probes a Fabry-Perot cavity whose resonance shows up as a
Lorentzian-shaped dip across the comb teeth; the comb is heterodyned against a
frequency-shifted local oscillator, so every tooth becomes one RF beat tone
that the digitiser samples.  The dip centre follows the proof-mass motion at the
mechanical resonance (23.686 kHz).

Synthesis recipe, one frame of N samples at sample rate fs:

* tooth i (0 <= i < K, optical order) is a cosine at integer bin k_i with
  amplitude A_i = b * (1 - d / (1 + (2 (i - c) / w)^2)) and phase pi i^2 / K;
* the frame is the exact sum of those cosines, built as an inverse real FFT
  of a spectrum holding (N/2) A_i exp(j phi_i) at bin k_i;
* white Gaussian noise of variance mean_t(s^2) / 10^(SNR/10);
* quantisation to `bits` bits, right-justified in int16, with a stream gain
  that maps 80 % of full scale onto the peak of the noiseless reference frame
  (unit teeth, no dip).

The centre moves as c(t) = c_mid + amp * sin(2 pi f_mech t) with t the start
time of the frame, or (learned warm-start data) every parameter sweeps its
range along a slow sinusoid; a per-frame uniform draw is also available.
Per-frame width, depth, SNR and tilt are drawn uniformly from the ranges in the
spec.  Random numbers come from numpy's PCG64 seeded by (seed, batch index),
so any batch of any stream is reproducible on its own.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Sequence, Tuple

import numpy as np

_F_MECH_HZ = 23_686.0


def tooth_bins_paper_c1() -> np.ndarray:
    """Beat bins |51 + 10 n| (n = -55 .. 44) at 1 MHz bin spacing.

    51 MHz local-oscillator shift and 10 MHz comb spacing (paper, Experimental
    Setup); with 1024-sample frames at 1.024 GS/s one bin is 1 MHz.  Optical
    order: tooth i has n = i - 55.
    """
    n = np.arange(-55, 45, dtype=np.int64)
    return np.abs(51 + 10 * n).astype(np.int32)


def tooth_bins_paper_2200() -> np.ndarray:
    """The paper's own comb: 220 teeth at beat frequencies |51 + 10 n| MHz,
    n = -115 .. 104, on the 1 MHz bins of 2200-sample frames at 2.2 GS/s
    (bins 1 .. 1099, all distinct: the two families end in 1 and in 9)."""
    n = np.arange(-115, 105)
    return np.abs(51 + 10 * n).astype(np.int32)


def tooth_bins_interleaved(n_samples: int, n_teeth: int) -> np.ndarray:
    """Two interleaved tooth families on distinct integer bins below Nyquist.

    A comb symmetric about the local oscillator folds into baseband as two
    families |b0 + s (i - h)|; h = ceil(K/2), s = floor((N/2 - 1)/(h + 1)),
    b0 = floor((s - 1)/2).  For N=2048, K=220 this gives s=9, b0=4, bins 4..986.
    """
    k = int(n_teeth)
    n = int(n_samples)
    h = (k + 1) // 2
    s = (n // 2 - 1) // (h + 1)
    if s < 2:
        raise ValueError(f"cannot place {k} teeth on distinct bins for N={n}")
    b0 = (s - 1) // 2
    i = np.arange(k, dtype=np.int64)
    bins = np.abs(b0 + s * (i - h))
    if len(np.unique(bins)) != k or bins.min() <= 0 or bins.max() >= n // 2:
        raise ValueError(f"interleaved layout collides for N={n}, K={k}")
    return bins.astype(np.int32)


@dataclass
class StreamSpec:
    """Parameters of one synthetic stream (all ranges are uniform [lo, hi])."""

    name: str
    n: int
    fs: float
    bins: np.ndarray
    f_mech: float = _F_MECH_HZ
    centre_mode: str = "sine"          # "sine", "uniform" or "drift"
    centre_amp: float = 10.0           # sine amplitude, teeth
    centre_halfrange: float = 40.0     # uniform mode: mid +- this
    centre_mid: Optional[float] = None  # default (K-1)/2
    width: Tuple[float, float] = (8.0, 8.0)
    depth: Tuple[float, float] = (0.6, 0.6)
    baseline: float = 1.0
    snr_db: Tuple[float, float] = (40.0, 40.0)
    tilt: Tuple[float, float] = (0.0, 0.0)
    bits: int = 14
    headroom: float = 0.8
    lineshape: str = "lorentzian"      # "lorentzian" or "fano"
    asym_q: float = float("inf")       # Fano asymmetry (fano lineshape only)
    power_drift: float = 0.0           # laser-power drift of the baseline, +- fraction
    power_drift_hz: float = 1700.0
    sample_dtype: str = "int16"        # "int16" or "int8" (then bits <= 8)

    @property
    def k(self) -> int:
        return int(len(self.bins))

    @property
    def mid(self) -> float:
        return (self.k - 1) / 2.0 if self.centre_mid is None else float(self.centre_mid)


@dataclass
class Batch:
    frames: np.ndarray        # int16 [F, N]
    ref_frames: np.ndarray    # int16 [R, N] noiseless unit-tooth reference frame(s)
    centre: np.ndarray        # float64 [F] true dip centre (teeth)
    width: np.ndarray         # float64 [F] true FWHM (teeth)
    depth: np.ndarray         # float64 [F]
    baseline: np.ndarray      # float64 [F]
    snr_db: np.ndarray        # float64 [F]
    tilt: np.ndarray          # float64 [F]
    gain: float               # counts per unit of tooth amplitude
    clipped: int              # samples that hit the converter rails
    first_frame: int = 0
    meta: dict = field(default_factory=dict)


def _phases(k: int) -> np.ndarray:
    i = np.arange(k, dtype=np.float64)
    return np.pi * i * i / k


def _synth(n: int, bins: np.ndarray, amps: np.ndarray, phases: np.ndarray) -> np.ndarray:
    """Exact sum of cosines A_i cos(2 pi k_i t / N + phi_i), one row per frame."""
    f = amps.shape[0]
    spec = np.zeros((f, n // 2 + 1), dtype=np.complex128)
    spec[:, bins] = (n / 2.0) * amps * np.exp(1j * phases)[None, :]
    return np.fft.irfft(spec, n=n, axis=1)


def _reference_float(spec: StreamSpec) -> np.ndarray:
    k = spec.k
    return _synth(spec.n, spec.bins, np.ones((1, k)), _phases(k))[0]


def stream_gain(spec: StreamSpec) -> float:
    full = 2 ** (spec.bits - 1) - 1
    return spec.headroom * full / float(np.max(np.abs(_reference_float(spec))))


def _quantise(x: np.ndarray, bits: int) -> Tuple[np.ndarray, int]:
    lo, hi = -(2 ** (bits - 1)), 2 ** (bits - 1) - 1
    q = np.rint(x)
    clipped = int(np.count_nonzero((q < lo) | (q > hi)))
    return np.clip(q, lo, hi).astype(np.int16), clipped


def _uniform(rng: np.random.Generator, rng_pair, size: int) -> np.ndarray:
    lo, hi = float(rng_pair[0]), float(rng_pair[1])
    u = rng.random(size)
    return lo + (hi - lo) * u


def make_batch(spec: StreamSpec, n_frames: int, seed: int, batch_index: int = 0,
               chunk: int = 4096, noise: bool = True, centre=None) -> Batch:
    """Generate `n_frames` consecutive frames of a stream.

    Batch b of a stream starts at frame b * n_frames, so consecutive batch
    indices continue the same time axis.  `noise=False` gives the quantised
    noiseless frames (used for closed-form checks).
    """
    n, k = spec.n, spec.k
    bins = np.asarray(spec.bins, dtype=np.int64)
    if bins.min() <= 0 or bins.max() >= n // 2:
        raise ValueError("tooth bins must lie strictly between DC and Nyquist")
    given = None if centre is None else np.asarray(centre, dtype=np.float64)
    rng = np.random.default_rng([int(seed), int(batch_index)])
    first = int(batch_index) * int(n_frames)
    f_idx = first + np.arange(n_frames, dtype=np.float64)
    t_start = f_idx * n / spec.fs

    width = _uniform(rng, spec.width, n_frames)
    depth = _uniform(rng, spec.depth, n_frames)
    snr = _uniform(rng, spec.snr_db, n_frames)
    tilt = _uniform(rng, spec.tilt, n_frames)
    if spec.centre_mode == "sine":
        centre = spec.mid + spec.centre_amp * np.sin(2.0 * np.pi * spec.f_mech * t_start)
    elif spec.centre_mode == "uniform":
        centre = _uniform(rng, (spec.mid - spec.centre_halfrange, spec.mid + spec.centre_halfrange),
                          n_frames)
    elif spec.centre_mode == "drift":
        # every parameter sweeps its range along a slow sinusoid (random rate and
        # phase per batch), so consecutive frames see a continuously moving dip
        def sweep(lo, hi, f_lo, f_hi):
            f = rng.uniform(f_lo, f_hi)
            ph = rng.uniform(0.0, 2.0 * np.pi)
            return lo + (hi - lo) * (0.5 + 0.5 * np.sin(2.0 * np.pi * f * t_start + ph))
        centre = sweep(spec.mid - spec.centre_halfrange, spec.mid + spec.centre_halfrange,
                       100.0, 800.0)
        width = sweep(spec.width[0], spec.width[1], 10.0, 200.0)
        depth = sweep(spec.depth[0], spec.depth[1], 10.0, 200.0)
        snr = sweep(spec.snr_db[0], spec.snr_db[1], 10.0, 200.0)
        tilt = sweep(spec.tilt[0], spec.tilt[1], 10.0, 200.0)
    else:
        raise ValueError(spec.centre_mode)
    if given is not None:
        # a given displacement series (teeth) in place of the spec's motion
        if given.shape != (n_frames,):
            raise ValueError("centre must hold one value per frame")
        centre = given
    baseline = np.full(n_frames, float(spec.baseline))
    if spec.power_drift:
        phase = rng.uniform(0.0, 2.0 * np.pi)
        baseline = baseline * (1.0 + spec.power_drift
                               * np.sin(2.0 * np.pi * spec.power_drift_hz * t_start + phase))

    gain = stream_gain(spec)
    phases = _phases(k)
    i = np.arange(k, dtype=np.float64)
    half = max((k - 1) / 2.0, 1.0)
    out = np.empty((n_frames, n), dtype=np.int16)
    clipped = 0
    for a in range(0, n_frames, chunk):
        b = min(n_frames, a + chunk)
        u = 2.0 * (i[None, :] - centre[a:b, None]) / width[a:b, None]
        if spec.lineshape == "fano":
            shape = (1.0 + u / spec.asym_q) ** 2 / (1.0 + u * u)
        else:
            shape = 1.0 / (1.0 + u * u)
        amps = baseline[a:b, None] * (1.0 - depth[a:b, None] * shape)
        amps = amps * (1.0 + tilt[a:b, None] * (i[None, :] - half) / half)
        s = _synth(n, bins, amps, phases)
        if noise:
            sigma = np.sqrt(np.mean(s * s, axis=1) / 10.0 ** (snr[a:b] / 10.0))
            s = s + sigma[:, None] * rng.standard_normal(s.shape)
        q, c = _quantise(gain * s, spec.bits)
        out[a:b] = q
        clipped += c

    ref, _ = _quantise(gain * _reference_float(spec)[None, :], spec.bits)
    if spec.sample_dtype == "int8":
        if spec.bits > 8:
            raise ValueError("int8 samples need bits <= 8")
        out = out.astype(np.int8)
        ref = ref.astype(np.int8)
    return Batch(frames=out, ref_frames=ref, centre=centre, width=width, depth=depth,
                 baseline=baseline, snr_db=snr, tilt=tilt, gain=gain, clipped=clipped,
                 first_frame=first, meta={"spec": spec.name, "seed": int(seed)})


def make_lorentzian_spectra(k: int, n_spectra: int, seed: int,
                            centre: Tuple[float, float], width: Tuple[float, float],
                            depth: Tuple[float, float], baseline: Tuple[float, float] = (1.0, 1.0),
                            sigma: Tuple[float, float] = (0.0, 0.0)):
    """Spectra y_i = b (1 - d / (1 + (2 (i - c)/w)^2)) + sigma * N(0,1), directly in
    the normalised tooth domain (no transform), with the true parameters."""
    rng = np.random.default_rng([int(seed), 7])
    c = _uniform(rng, centre, n_spectra)
    w = _uniform(rng, width, n_spectra)
    d = _uniform(rng, depth, n_spectra)
    b = _uniform(rng, baseline, n_spectra)
    s = _uniform(rng, sigma, n_spectra)
    i = np.arange(k, dtype=np.float64)
    u = 2.0 * (i[None, :] - c[:, None]) / w[:, None]
    y = b[:, None] * (1.0 - d[:, None] / (1.0 + u * u))
    y = y + s[:, None] * rng.standard_normal(y.shape)
    truth = np.stack([c, w, d, b], axis=1)
    return y, truth, s


# ---------------------------------------------------------------------------
# The five workloads.
# ---------------------------------------------------------------------------

def spec_tiny() -> StreamSpec:
    """4096 x 1024-sample frames at 1.024 GS/s, 100 teeth |51+10n|, FWHM 8,
    depth 0.6, centre +-10 teeth at 23.686 kHz, 40 dB SNR, 14 bit."""
    return StreamSpec(name="tiny", n=1024, fs=1.024e9, bins=tooth_bins_paper_c1(),
                      width=(8.0, 8.0), depth=(0.6, 0.6), snr_db=(40.0, 40.0))


def spec_paper_rate() -> StreamSpec:
    """2048-sample frames at 1.1 GS/s (2.2 GB/s of int16), 220 teeth,
    per-frame FWHM U[4,16] teeth and SNR U[20,50] dB."""
    return StreamSpec(name="paper_rate", n=2048, fs=1.1e9, bins=tooth_bins_interleaved(2048, 220),
                      width=(4.0, 16.0), depth=(0.6, 0.6), snr_db=(20.0, 50.0))


def spec_precision() -> StreamSpec:
    """As the paper-rate stream with 4096-sample frames."""
    return StreamSpec(name="precision", n=4096, fs=1.1e9, bins=tooth_bins_interleaved(4096, 220),
                      width=(4.0, 16.0), depth=(0.6, 0.6), snr_db=(20.0, 50.0))


def spec_learned() -> StreamSpec:
    """Warm-start training distribution: centre mid+-40, FWHM 3..20, depth
    0.1..0.9, SNR 15..50 dB, linear baseline tilt +-5%, each swept along a
    slow sinusoid (centre at 100-800 Hz, the others at 10-200 Hz) so the dip
    moves continuously from frame to frame."""
    return StreamSpec(name="learned", n=2048, fs=1.1e9, bins=tooth_bins_interleaved(2048, 220),
                      centre_mode="drift", centre_halfrange=40.0, width=(3.0, 20.0),
                      depth=(0.1, 0.9), snr_db=(15.0, 50.0), tilt=(-0.05, 0.05))


def spec_fano() -> StreamSpec:
    """The paper's own lineshape at the paper rate: 2048-sample frames at
    1.1 GS/s, 220 teeth, an asymmetric Fano dip of fixed width 8.03 teeth
    (the cavity linewidth: free spectral range over finesse, in 10 MHz
    teeth) and asymmetry q = 4, depth 0.6, the baseline following a +-5 %
    laser-power drift at 1.7 kHz, centre +-10 teeth at 23.686 kHz, SNR
    U[20,50] dB."""
    return StreamSpec(name="fano", n=2048, fs=1.1e9, bins=tooth_bins_interleaved(2048, 220),
                      width=(8.03, 8.03), depth=(0.6, 0.6), snr_db=(20.0, 50.0),
                      lineshape="fano", asym_q=4.0, power_drift=0.05)


def spec_paper8() -> StreamSpec:
    """The paper's own ingest geometry: 8-bit samples at 2.2 GS/s in
    2200-sample (1 us) frames, 220 teeth at |51 + 10 n| MHz (n = -115..104)
    on 1 MHz bins, with the Fano dip of spec_fano (fixed width 8.03 teeth,
    asymmetry 4, depth 0.6, +-5 % laser-power drift), centre +-10 teeth at
    23.686 kHz, SNR U[20,50] dB before the 8-bit quantisation."""
    return StreamSpec(name="paper8", n=2200, fs=2.2e9, bins=tooth_bins_paper_2200(),
                      width=(8.03, 8.03), depth=(0.6, 0.6), snr_db=(20.0, 50.0),
                      lineshape="fano", asym_q=4.0, power_drift=0.05, bits=8,
                      sample_dtype="int8")


def spec_multistream(seed: int = 100, n_streams: int = 16) -> Sequence[StreamSpec]:
    """16 streams with frame lengths cycling over 512..8192 and K_s drawn from
    64..min(440, N_s/4); per stream FWHM U[4,16], depth U[0.3,0.8], SNR
    U[20,50] dB and mechanical frequency 23.686 kHz * U[0.9, 1.1]."""
    lengths = [512, 1024, 2048, 4096, 8192]
    rng = np.random.default_rng([int(seed), 99])
    out = []
    for s in range(n_streams):
        n = lengths[s % len(lengths)]
        kmax = min(440, n // 4)
        k = int(rng.integers(64, kmax + 1))
        w = float(rng.uniform(4.0, 16.0))
        d = float(rng.uniform(0.3, 0.8))
        snr = float(rng.uniform(20.0, 50.0))
        fm = _F_MECH_HZ * float(rng.uniform(0.9, 1.1))
        out.append(StreamSpec(name=f"stream{s:02d}", n=n, fs=1.1e9,
                              bins=tooth_bins_interleaved(n, k), f_mech=fm,
                              width=(w, w), depth=(d, d), snr_db=(snr, snr)))
    return out


def make_displacement(n: int, fs: float, f0: float, q: float, drive: float, floor: float,
                      drift: float, seed: int, chunk: int = 1 << 22) -> np.ndarray:
    """A displacement series (teeth) as the fitted centres of a still
    accelerometer would give it: the thermomechanical resonance (a damped
    oscillator driven by white force noise, integrated exactly at the frame
    rate as the second-order recursion x[t] = a1 x[t-1] + a2 x[t-2] + e[t],
    poles r e^{+-i theta}, r = exp(-pi f0 / (Q fs)), theta = 2 pi f0
    sqrt(1 - 1/(4 Q^2)) / fs, e white with deviation `drive`), a white
    measurement floor of deviation `floor` (the centre fit's noise) and a slow
    random-walk drift of step deviation `drift` (thermal and humidity
    drifts).  float32 [n]."""
    from scipy.signal import lfilter
    rng = np.random.default_rng([int(seed), 11])
    r = np.exp(-np.pi * f0 / (q * fs))
    theta = 2.0 * np.pi * f0 * np.sqrt(1.0 - 1.0 / (4.0 * q * q)) / fs
    a1, a2 = 2.0 * r * np.cos(theta), -r * r
    out = np.empty(n, dtype=np.float32)
    zi = np.zeros(2)
    walk = 0.0
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        e = drive * rng.standard_normal(b - a)
        x, zi = lfilter([1.0], [1.0, -a1, -a2], e, zi=zi)
        steps = np.cumsum(drift * rng.standard_normal(b - a)) + walk
        walk = float(steps[-1])
        out[a:b] = x + steps + floor * rng.standard_normal(b - a)
    return out
