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
