"""Comparison helpers for the GPU parity tests (test code, not product code).

Bars
----
* raw tooth amplitudes: relative error <= 1e-4 against the FP64 oracle, on
  bins that carry a comb tooth (all synthetic teeth do); for arbitrary input
  bins the error is measured against the RMS amplitude of the frame instead;
* start point: bit-identical to the oracle when both see the same float32
  normalised spectra (every value is an exact selection or an IEEE float32
  operation taken in the same order);
* fitted centre: |c_gpu - c_oracle| <= 1e-3 * FWHM_oracle on frames where the
  oracle converged.  A mismatch is exempt when the two fits are equally good
  minima: chi2 re-evaluated in FP64 at the GPU parameters is within
  (1 + 1e-6) of the oracle's chi2.  The fraction meeting the bar (after
  exemptions) must be >= 99.9 %.
"""

import numpy as np

import oracle

MAG_RTOL = 1e-4
CENTRE_FWHM_TOL = 1e-3
PASS_FRACTION = 0.999


def mag_rel_err(gpu, ora):
    gpu = np.asarray(gpu, dtype=np.float64)
    ora = np.asarray(ora, dtype=np.float64)
    return np.abs(gpu - ora) / np.maximum(np.abs(ora), 1e-300)


def warm_compared(status):
    """Statuses for centre_parity on the warm path: both sides run the same
    short polish, so a frame is compared whether the polish converged (0),
    stopped at its iteration cap (1) or fell back to the cold fit (3); only a
    singular fit (2) is left out."""
    st = np.asarray(status)
    return np.where(st == 2, 2, 0)


def full_fit_compared(status):
    """Statuses for centre_parity on the warm path when the polish runs to the
    cold start's cap (a full LM fit from the network's start point): as for
    the cold path, frames whose fit stopped at the cap (1) or was singular (2)
    are left out, since a fit that has not converged has no unique end point
    (in ill-conditioned valleys it depends on rounding along the path);
    converged fits (0) and cold refits (3) are compared."""
    st = np.asarray(status)
    return np.where(st == 3, 0, st)


def centre_parity(y_oracle, p_gpu, p_oracle, st_oracle, chi2_oracle):
    """Returns dict with fraction passing, exemptions and the outlier rows."""
    p_gpu = np.asarray(p_gpu, dtype=np.float64)
    p_oracle = np.asarray(p_oracle, dtype=np.float64)
    conv = np.asarray(st_oracle) == 0
    err = np.abs(p_gpu[:, 0] - p_oracle[:, 0]) / np.abs(p_oracle[:, 1])
    ok = err <= CENTRE_FWHM_TOL
    exempt = np.zeros_like(ok)
    for f in np.nonzero(conv & ~ok)[0]:
        if np.all(np.isfinite(p_gpu[f])) and p_gpu[f, 1] > 0:
            c2 = oracle.chi2_at(y_oracle[f], p_gpu[f])
            exempt[f] = c2 <= chi2_oracle[f] * (1.0 + 1e-6)
    n = int(conv.sum())
    good = int((ok | exempt)[conv].sum())
    return {"n": n, "fraction": good / max(n, 1), "exempt": int(exempt[conv].sum()),
            "outliers": np.nonzero(conv & ~ok & ~exempt)[0], "max_err": float(err[conv].max())
            if n else 0.0}
