"""Ingest, DFT at the tooth bins, magnitude and reference average (FP64).

Test infrastructure only (see the package docstring).

Paper, Data Capture and Processing: the integer samples are cast to floating
point, the 1-D stream is reshaped into rows of consecutive samples (one frame
per row), each row is Fourier transformed, and the bins of the comb teeth are
picked out in optical order.

Readings taken where the paper is silent or garbled:
* the transform is the forward, unnormalised DFT of a real row,
  X[k] = sum_t x[t] exp(-2 pi i k t / N); the paper calls it a complex-to-real
  FFT, which cannot apply to real samples;
* what is kept per tooth is the amplitude |X[k_i]|;
* the reference spectrum is the arithmetic mean of per-frame amplitudes.

An FFT computes this DFT exactly up to rounding, so the oracle is the DFT
definition itself: the sum over t written as a matrix product against the
explicit cos/sin basis, with the phase index k t reduced modulo N in integer
arithmetic before the FP64 multiply.
"""

import numpy as np


def frames_to_float(frames) -> np.ndarray:
    """Cast integer frames [F, N] (int16, or the paper's int8) to float64
    (exact)."""
    x = np.asarray(frames)
    if x.dtype not in (np.int16, np.int8):
        raise TypeError(f"frames must be int16 or int8, got {x.dtype}")
    if x.ndim != 2:
        raise ValueError("frames must be [n_frames, frame_len]")
    return x.astype(np.float64)


def _basis(n: int, bins) -> tuple:
    t = np.arange(n, dtype=np.int64)
    k = np.asarray(bins, dtype=np.int64)
    phase = np.outer(t, k) % n               # exact integer reduction of k t mod N
    theta = (2.0 * np.pi / n) * phase.astype(np.float64)
    return np.cos(theta), np.sin(theta)


def dft_at_bins(frames, bins, chunk: int = 8192):
    """X_f[k_i] = sum_t x_f[t] (cos(2 pi k_i t/N) - i sin(2 pi k_i t/N)).

    Returns (re, im) float64 arrays [F, K].
    """
    x = frames_to_float(frames)
    cos_b, sin_b = _basis(x.shape[1], bins)
    re = np.empty((x.shape[0], cos_b.shape[1]))
    im = np.empty_like(re)
    for a in range(0, x.shape[0], chunk):
        b = min(x.shape[0], a + chunk)
        re[a:b] = x[a:b] @ cos_b
        im[a:b] = -(x[a:b] @ sin_b)
    return re, im


def tooth_magnitudes(frames, bins) -> np.ndarray:
    """m_f,i = |X_f[k_i]|, float64 [F, K]."""
    re, im = dft_at_bins(frames, bins)
    return np.hypot(re, im)


def reference_spectrum(ref_frames, bins) -> np.ndarray:
    """Mean over the reference frames of the tooth amplitudes, float64 [K]."""
    return tooth_magnitudes(ref_frames, bins).mean(axis=0)


def full_dft(frame) -> np.ndarray:
    """All N/2+1 bins of one frame by the same definition (used for checks)."""
    f = np.asarray(frame).reshape(1, -1)
    n = f.shape[1]
    re, im = dft_at_bins(f, np.arange(n // 2 + 1))
    return re[0] + 1j * im[0]
