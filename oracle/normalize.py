"""Division of each spectrum by the reference spectrum (FP64).

Test infrastructure only (see the package docstring).

Paper, Data Capture and Processing: each row of tooth amplitudes is divided by
a previously computed average reference spectrum, giving the normalised cavity
spectra.  Reading: a plain linear ratio (no logarithm), with a strictly
positive, finite reference.
"""

import numpy as np


def normalize(mags, ref) -> np.ndarray:
    """y_f,i = m_f,i / ref_i."""
    m = np.asarray(mags, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    if r.ndim != 1 or m.shape[-1] != r.shape[0]:
        raise ValueError("reference length must equal the number of teeth")
    if not np.all(np.isfinite(r)) or np.any(r <= 0):
        raise ValueError("reference must be finite and > 0")
    return m / r[None, :]
