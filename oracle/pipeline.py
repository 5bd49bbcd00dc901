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
from .lm import lm_fit_batch


def process_batch(frames, bins, ref, max_iter: int = 20, tol: float = 1e-6):
    """Returns a dict with mags [F,K], y [F,K], p0 [F,4], params [F,4],
    iters [F], status [F], chi2 [F]."""
    mags = tooth_magnitudes(frames, bins)
    y = normalize(mags, ref)
    p0 = initial_guess(y)
    params, iters, status, chi2 = lm_fit_batch(y, p0, max_iter, tol)
    return {"mags": mags, "y": y, "p0": p0, "params": params, "iters": iters,
            "status": status, "chi2": chi2}


def process_batch_warm(frames, bins, ref, params, out_mean, out_std, noise_floor,
                       polish_iter: int = 2, max_iter: int = 20, tol: float = 1e-6):
    """Learned warm start: network start point (bfloat16 operands emulated),
    a short LM polish, and the cold-start fit for frames whose RMS residual
    sqrt(chi2/(K-4)) exceeds 2 * noise_floor (status 3)."""
    from . import mlp
    from .lm import lm_fit
    mags = tooth_magnitudes(frames, bins)
    y = normalize(mags, ref)
    k = y.shape[1]
    x = mlp.resample_to_input(y.astype(np.float32).astype(np.float64))
    z, _ = mlp.forward(x, params, bf16_ops=True)
    p0 = z * np.asarray(out_std, dtype=np.float64) + np.asarray(out_mean, dtype=np.float64)
    p0[:, :2] *= (k - 1) / (mlp.IN - 1)
    cold_p0 = None
    f_count = y.shape[0]
    params_out = np.empty((f_count, 4))
    iters = np.empty(f_count, dtype=np.int32)
    status = np.empty(f_count, dtype=np.int32)
    chi2 = np.empty(f_count)
    thr2 = 4.0 * noise_floor ** 2 * max(k - 4, 1)
    for f in range(f_count):
        p, it, st, c2 = lm_fit(y[f], p0[f], polish_iter, tol)
        if not np.isfinite(c2) or c2 > thr2:
            if cold_p0 is None:
                cold_p0 = initial_guess(y)
            p, it, st, c2 = lm_fit(y[f], cold_p0[f], max_iter, tol)
            st = 3
        params_out[f], iters[f], status[f], chi2[f] = p, it, st, c2
    return {"mags": mags, "y": y, "p0": p0, "params": params_out, "iters": iters,
            "status": status, "chi2": chi2}
