"""Displacement power spectral density and the mechanical resonance fit (FP64).

Test infrastructure only (see the package docstring).

Paper, Experimental Results and the figure of the power spectral density: the
fitted cavity centres form a displacement time series (one value per frame);
its power spectral density, averaged over 1 s, 10 s and 10 min of data, shows
the accelerometer's thermomechanical resonance near 24 kHz, and a fit of that
resonance gives the mechanical resonance frequency f and quality factor Q.

Readings (the paper names neither the estimator nor the fitted model):
* Welch's averaged periodogram: segments of L samples (L = 2^16 by default)
  overlapping by L/2, the segment mean removed, a periodic Hann window
  w[t] = (1 - cos(2 pi t / L)) / 2, one-sided density
      P[k] = (2 / (fs sum_t w[t]^2)) |sum_t w[t] (x[t] - mean) e^{-2 pi i k t / L}|^2
  (factor 1 instead of 2 at k = 0 and k = L/2), averaged over the segments;
  only a band of bins around the resonance is evaluated;
* the resonance: a harmonic oscillator driven by white force noise plus a
  white measurement floor,
      S(f) = A / ((f0^2 - f^2)^2 + (f0 f / Q)^2) + B,
  fitted by least squares on the logarithm (the Welch estimate's scatter is
  relative), parameters p = (ln A, f0, Q, ln B), by Levenberg-Marquardt with
  the plain fit's schedule (lam0 = 1e-3, /10 on accept, *10 on reject,
  Cholesky), at most `max_iter` iterations, converged when an accepted step
  lowers chi2 by at most tol * chi2, tol = 1e-9 by default (a tighter one
  drives the damping so low on a measured spectrum that the normal matrix of
  the four strongly correlated parameters stops being numerically positive
  definite, after the parameters have settled far below their statistical
  uncertainty);
* start point: f0 at the largest band value; B the median of the band's
  lowest quarter of values; Q = f0 / (the width between the first bins on
  each side of the peak whose excess over B falls to half the peak's), at
  least 1; A from S(f0) = A Q^2 / f0^4 + B.
"""

import numpy as np

from .lm import STATUS_CONVERGED, STATUS_MAX_ITER, STATUS_SINGULAR


def hann(seg_len):
    t = np.arange(seg_len, dtype=np.float64)
    return 0.5 - 0.5 * np.cos(2.0 * np.pi * t / seg_len)


def welch_band(x, fs, seg_len, k_lo, n_bins):
    """One-sided Welch density at bins k_lo .. k_lo + n_bins - 1 (float64)."""
    x = np.asarray(x, dtype=np.float64)
    hop = seg_len // 2
    n_seg = (x.shape[0] - seg_len) // hop + 1
    if n_seg < 1:
        raise ValueError("series shorter than one segment")
    w = hann(seg_len)
    k = np.arange(k_lo, k_lo + n_bins, dtype=np.int64)
    t = np.arange(seg_len, dtype=np.int64)
    phase = (np.outer(t, k) % seg_len).astype(np.float64) * (2.0 * np.pi / seg_len)
    cos_b, sin_b = np.cos(phase), np.sin(phase)
    acc = np.zeros(n_bins)
    for s in range(n_seg):
        seg = x[s * hop:s * hop + seg_len]
        v = (seg - seg.mean()) * w
        re = v @ cos_b
        im = -(v @ sin_b)
        acc += re * re + im * im
    scale = 2.0 / (fs * float(w @ w))
    edge = (k == 0) | (k == seg_len // 2)
    dens = acc / n_seg * scale
    dens[edge] *= 0.5
    return dens


def oscillator(f, p):
    la, f0, q, lb = (float(v) for v in p)
    f = np.asarray(f, dtype=np.float64)
    return np.exp(la) / ((f0 * f0 - f * f) ** 2 + (f0 * f / q) ** 2) + np.exp(lb)


def oscillator_log_jacobian(f, p):
    """Partial derivatives of ln S with respect to (ln A, f0, Q, ln B)."""
    la, f0, q, lb = (float(v) for v in p)
    f = np.asarray(f, dtype=np.float64)
    den = (f0 * f0 - f * f) ** 2 + (f0 * f / q) ** 2
    res = np.exp(la) / den
    s = res + np.exp(lb)
    dden_df0 = 4.0 * f0 * (f0 * f0 - f * f) + 2.0 * f0 * f * f / (q * q)
    dden_dq = -2.0 * f0 * f0 * f * f / (q * q * q)
    jac = np.empty((f.shape[0], 4))
    jac[:, 0] = res / s
    jac[:, 1] = -res * dden_df0 / den / s
    jac[:, 2] = -res * dden_dq / den / s
    jac[:, 3] = np.exp(lb) / s
    return jac


def start_point(freqs, psd):
    psd = np.asarray(psd, dtype=np.float64)
    f = np.asarray(freqs, dtype=np.float64)
    i = int(np.argmax(psd))
    b = float(np.median(np.sort(psd)[:max(1, psd.shape[0] // 4)]))
    half = b + 0.5 * (psd[i] - b)
    lo = i
    while lo > 0 and psd[lo] > half:
        lo -= 1
    hi = i
    while hi < psd.shape[0] - 1 and psd[hi] > half:
        hi += 1
    f0 = f[i]
    width = max(f[hi] - f[lo], f[1] - f[0])
    q = max(1.0, f0 / width)
    a = max(psd[i] - b, 1e-300) * f0 ** 4 / (q * q)
    return np.array([np.log(a), f0, q, np.log(max(b, 1e-300))])


def oscillator_fit(freqs, psd, p0=None, max_iter: int = 100, tol: float = 1e-9,
                   lam0: float = 1e-3):
    """Returns (p = (ln A, f0, Q, ln B), iterations, status, chi2)."""
    f = np.asarray(freqs, dtype=np.float64)
    ly = np.log(np.asarray(psd, dtype=np.float64))
    p = start_point(f, psd) if p0 is None else np.asarray(p0, dtype=np.float64).copy()
    r = ly - np.log(oscillator(f, p))
    chi2 = float(r @ r)
    jac = oscillator_log_jacobian(f, p)
    a = jac.T @ jac
    g = jac.T @ r
    lam = lam0
    status = STATUS_MAX_ITER
    it = 0
    while it < max_iter:
        it += 1
        try:
            low = np.linalg.cholesky(a + lam * np.diag(np.diag(a)))
        except np.linalg.LinAlgError:
            status = STATUS_SINGULAR
            break
        delta = np.linalg.solve(low.T, np.linalg.solve(low, g))
        trial = p + delta
        ok = bool(np.all(np.isfinite(trial))) and trial[1] > 0 and trial[2] > 0
        if ok:
            r_t = ly - np.log(oscillator(f, trial))
            chi2_t = float(r_t @ r_t)
            ok = np.isfinite(chi2_t) and chi2_t <= chi2
        if not ok:
            lam *= 10.0
            continue
        drop = chi2 - chi2_t
        old = chi2
        p, chi2 = trial, chi2_t
        jac = oscillator_log_jacobian(f, p)
        a = jac.T @ jac
        g = jac.T @ r_t
        lam /= 10.0
        if drop <= tol * old:
            status = STATUS_CONVERGED
            break
    return p, it, status, chi2
