"""The oracle's steps chained for one batch of frames.

Test infrastructure only (see the package docstring).

Order as in the paper's processing description and figure: cast and frame,
transform, pick the teeth, divide by the reference, median-filter start point,
Levenberg-Marquardt fit.
"""

import numpy as np

from .dft import tooth_magnitudes
from .normalize import normalize
from .initializer import initial_guess
from .lm import lm_fit, lm_fit_batch

STATUS_FALLBACK = 3


def process_batch(frames, bins, ref, max_iter: int = 20, tol: float = 1e-6):
    """Returns a dict with mags [F,K], y [F,K], p0 [F,4], params [F,4],
    iters [F], status [F], chi2 [F]."""
    mags = tooth_magnitudes(frames, bins)
    y = normalize(mags, ref)
    p0 = initial_guess(y)
    params, iters, status, chi2 = lm_fit_batch(y, p0, max_iter, tol)
    return {"mags": mags, "y": y, "p0": p0, "params": params, "iters": iters,
            "status": status, "chi2": chi2}


def process_batch_fano(frames, bins, ref, width, q, dbar, bbar, max_iter: int = 20,
                       tol: float = 1e-6, rows=None):
    """The paper's own fit for a batch: transform, teeth, reference division,
    7x7-median start centres, and the box-constrained LM fit of the Fano dip
    with width and asymmetry fixed and extent and scale within +-10 % of the
    averages dbar, bbar (every frame, or `rows`)."""
    from .fano import fano_box, fano_fit_batch
    mags = tooth_magnitudes(frames, bins)
    y = normalize(mags, ref)
    p0 = initial_guess(y)
    params, iters, status, chi2 = fano_fit_batch(y, p0[:, 0], width, q, dbar, bbar, max_iter,
                                                 tol, rows)
    return {"mags": mags, "y": y, "p0": p0, "box": fano_box(dbar, bbar), "params": params,
            "iters": iters, "status": status, "chi2": chi2}


def network_start(y, params, out_mean, out_std):
    """Start points of the learned warm start for spectra y [F, K]: the
    network's standardised outputs z mapped to p = z * std + mean, computed on
    y resampled onto the network's 220 inputs; for K != 220 the centre and
    width (tooth units) are scaled by (K - 1) / 219.  The spectra enter the
    network as float32 values (bfloat16 operand rounding emulated)."""
    from . import mlp
    y = np.asarray(y, dtype=np.float64)
    k = y.shape[1]
    x = mlp.resample_to_input(y.astype(np.float32).astype(np.float64))
    z, _ = mlp.forward(x, params, bf16_ops=True)
    p0 = z * np.asarray(out_std, dtype=np.float64) + np.asarray(out_mean, dtype=np.float64)
    p0[:, :2] *= (k - 1) / (mlp.IN - 1)
    return p0


def warm_fit(y, p0, noise_floor, polish_iter: int = 2, max_iter: int = 20, tol: float = 1e-6,
             rows=None):
    """Polish each spectrum from its warm start point p0 by `polish_iter` LM
    iterations; a frame whose RMS residual sqrt(chi2 / (K - 4)) then exceeds
    2 * noise_floor (or is not finite) is fitted again from the cold start
    point (7x7 median over the whole batch y) with up to `max_iter`
    iterations and gets status 3.  Its reported iteration count is the
    refit's.  With `rows`, only those frames of y are fitted (p0 then holds
    their start points, in that order).  Returns (params, iters, status,
    chi2, fell_back) for the fitted frames."""
    y = np.asarray(y, dtype=np.float64)
    k = y.shape[1]
    rows = np.arange(y.shape[0]) if rows is None else np.asarray(rows)
    f_count = rows.shape[0]
    cold_p0 = None
    params_out = np.empty((f_count, 4))
    iters = np.empty(f_count, dtype=np.int32)
    status = np.empty(f_count, dtype=np.int32)
    chi2 = np.empty(f_count)
    fell = np.zeros(f_count, dtype=bool)
    # RMS residual > 2 sigma  <=>  chi2 > 4 sigma^2 (K - 4)
    thr2 = 4.0 * noise_floor ** 2 * max(k - 4, 1)
    for j, f in enumerate(rows):
        p, it, st, c2 = lm_fit(y[f], p0[j], polish_iter, tol)
        if not np.isfinite(c2) or c2 > thr2:
            if cold_p0 is None:
                cold_p0 = initial_guess(y)
            p, it, st, c2 = lm_fit(y[f], cold_p0[f], max_iter, tol)
            st = STATUS_FALLBACK
            fell[j] = True
        params_out[j], iters[j], status[j], chi2[j] = p, it, st, c2
    return params_out, iters, status, chi2, fell


def process_batch_warm(frames, bins, ref, params, out_mean, out_std, noise_floor,
                       polish_iter: int = 2, max_iter: int = 20, tol: float = 1e-6):
    """Learned warm start for a batch of frames: transform, teeth, reference
    division, network start point, short LM polish, cold-start refit of the
    frames the residual test rejects (status 3)."""
    mags = tooth_magnitudes(frames, bins)
    y = normalize(mags, ref)
    p0 = network_start(y, params, out_mean, out_std)
    params_out, iters, status, chi2, _ = warm_fit(y, p0, noise_floor, polish_iter, max_iter, tol)
    return {"mags": mags, "y": y, "p0": p0, "params": params_out, "iters": iters,
            "status": status, "chi2": chi2}
