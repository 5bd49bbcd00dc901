"""Projected Levenberg-Marquardt fit of the asymmetric Fano cavity dip (FP64).

Test infrastructure only (see the package docstring).

Paper, Data Capture and Processing: each spectrum is fitted with a
five-parameter asymmetric Fano lineshape by Levenberg-Marquardt (at most 20
iterations, tolerance 1e-6).  Only the centre is free; the two parameters
for the scale and the extent of the peak are held within about +-10 % of a
pre-computed average value; the asymmetry and the width are fixed to values
measured beforehand for the device.  The figure on the GPU processing adds
that the spectra are averaged over space and time to set the initial
parameters.

Readings taken where the paper is silent:
* lineshape (q -> infinity gives the Lorentzian dip of the plain path):

      f(x; c, w, d, b, q) = b (1 - d (1 + u / q)^2 / (1 + u^2)),  u = 2 (x - c) / w,

  with c the centre, w the width and q the asymmetry (both fixed), d the
  extent (depth) and b the scale (baseline level, which follows the laser
  power);
* the deepest point of the dip lies at u = 1 / q with depth d (1 + 1/q^2);
* the box: d in [0.9, 1.1] dbar and b in [0.9, 1.1] bbar, where dbar and
  bbar are the pre-calculated averages, taken as inputs measured beforehand
  for the device like w and q (the 7x7-median start point underestimates a
  dip only a few teeth wide, so averages of it would put the box beside the
  dip);
* start point: the centre of the 7x7 median initializer of the plain path
  (lowest filtered value) and the averages dbar, bbar for the boxed
  parameters (the figure on GPU processing: averaged spectra set the initial
  parameters);
* the free parameters (c, d, b) are fitted by the damped normal equations of
  the plain path's schedule (lam0 = 1e-3, /10 on accept, *10 on reject,
  Cholesky, accept when finite and chi2 does not increase, converged when an
  accepted step lowers chi2 by at most tol * chi2 or chi2 <= 1e-30, status 2
  when the damped matrix is not positive definite), with the box kept by an
  active set: a boxed parameter that sits on a bound while chi2 would fall
  by moving it out of the box (J^T r pointing outward) is held for that
  step (its row and column of the damped system are replaced by the
  identity and its right-hand side by 0), and every trial point is projected
  onto the box before it is evaluated.  Converged, the fit is the minimum of
  chi2 over the box (the Karush-Kuhn-Tucker point).
"""

import numpy as np

from .lm import STATUS_CONVERGED, STATUS_MAX_ITER, STATUS_SINGULAR

BOX_HALF = 0.10


def fano(x, c, w, d, b, q):
    u = 2.0 * (np.asarray(x, dtype=np.float64) - c) / w
    return b * (1.0 - d * (1.0 + u / q) ** 2 / (1.0 + u * u))


def fano_jacobian(x, c, w, d, b, q):
    """Partial derivatives [K, 3] with respect to (c, d, b).

    With u = 2 (x - c)/w, D = 1 + u^2, s = 1 + u/q and g = s^2 / D:
      dg/du = (2 s / q) / D - 2 u s^2 / D^2,
      df/dc = -b d dg/du du/dc = (2 b d / w) dg/du,
      df/dd = -b g,   df/db = 1 - d g.
    """
    x = np.asarray(x, dtype=np.float64)
    u = 2.0 * (x - c) / w
    den = 1.0 + u * u
    s = 1.0 + u / q
    g = s * s / den
    dg_du = (2.0 * s / q) / den - 2.0 * u * s * s / (den * den)
    jac = np.empty((x.shape[0], 3))
    jac[:, 0] = (2.0 * b * d / w) * dg_du
    jac[:, 1] = -b * g
    jac[:, 2] = 1.0 - d * g
    return jac


def chi2_fano(y, c, w, d, b, q):
    y = np.asarray(y, dtype=np.float64)
    r = y - fano(np.arange(y.shape[0]), c, w, d, b, q)
    return float(r @ r)


def fano_box(dbar, bbar):
    """Box of the extent and scale, [[d_lo, d_hi], [b_lo, b_hi]]: +-10 % of
    the pre-calculated averages."""
    return np.array([[(1.0 - BOX_HALF) * dbar, (1.0 + BOX_HALF) * dbar],
                     [(1.0 - BOX_HALF) * bbar, (1.0 + BOX_HALF) * bbar]])


def _project(c, d, b, box):
    (dlo, dhi), (blo, bhi) = box
    return c, min(max(d, dlo), dhi), min(max(b, blo), bhi)


def _cholesky_solve(a, g):
    try:
        low = np.linalg.cholesky(a)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(low)):
        return None
    return np.linalg.solve(low.T, np.linalg.solve(low, g))


def fano_fit(y, p0, w, q, box, max_iter: int = 20, tol: float = 1e-6, lam0: float = 1e-3):
    """Fit (c, d, b) of one spectrum from p0 = (c0, d0, b0) (projected into
    the box first).  Returns ((c, d, b), iterations, status, chi2)."""
    y = np.asarray(y, dtype=np.float64)
    x = np.arange(y.shape[0], dtype=np.float64)
    c, d, b = _project(*(float(v) for v in p0), box)
    r = y - fano(x, c, w, d, b, q)
    chi2 = float(r @ r)
    if not np.isfinite(chi2):
        return np.array([c, d, b]), 0, STATUS_SINGULAR, chi2
    if chi2 <= 1e-30:
        return np.array([c, d, b]), 0, STATUS_CONVERGED, chi2
    jac = fano_jacobian(x, c, w, d, b, q)
    a = jac.T @ jac
    g = jac.T @ r
    lam = lam0
    status = STATUS_MAX_ITER
    it = 0
    while it < max_iter:
        it += 1
        damped = a + lam * np.diag(np.diag(a))
        rhs = g.copy()
        for j, (lo, hi) in ((1, box[0]), (2, box[1])):
            v = (d, b)[j - 1]
            if (v <= lo and g[j] < 0.0) or (v >= hi and g[j] > 0.0):
                damped[j, :] = 0.0
                damped[:, j] = 0.0
                damped[j, j] = 1.0
                rhs[j] = 0.0
        delta = _cholesky_solve(damped, rhs)
        if delta is None:
            status = STATUS_SINGULAR
            break
        tc, td, tb = _project(c + delta[0], d + delta[1], b + delta[2], box)
        ok = bool(np.isfinite(tc) and np.isfinite(td) and np.isfinite(tb))
        if ok:
            r_t = y - fano(x, tc, w, td, tb, q)
            chi2_t = float(r_t @ r_t)
            ok = np.isfinite(chi2_t) and chi2_t <= chi2
        if not ok:
            lam *= 10.0
            continue
        drop = chi2 - chi2_t
        old = chi2
        c, d, b, chi2 = tc, td, tb, chi2_t
        jac = fano_jacobian(x, c, w, d, b, q)
        a = jac.T @ jac
        g = jac.T @ r_t
        lam /= 10.0
        if drop <= tol * old or chi2 <= 1e-30:
            status = STATUS_CONVERGED
            break
    return np.array([c, d, b]), it, status, chi2


def fano_fit_batch(y, c0, w, q, dbar, bbar, max_iter: int = 20, tol: float = 1e-6, rows=None):
    """Fit rows of y [F, K] from start centres c0 [F] and the averages
    (dbar, bbar); returns params [F', 4] as (c, w, d, b), iters, status,
    chi2 for the fitted rows (all, or `rows`)."""
    y = np.asarray(y, dtype=np.float64)
    c0 = np.asarray(c0, dtype=np.float64)
    box = fano_box(dbar, bbar)
    rows = np.arange(y.shape[0]) if rows is None else np.asarray(rows)
    out = np.empty((rows.shape[0], 4))
    iters = np.empty(rows.shape[0], dtype=np.int32)
    status = np.empty(rows.shape[0], dtype=np.int32)
    chi2 = np.empty(rows.shape[0])
    for j, f in enumerate(rows):
        (c, d, b), iters[j], status[j], chi2[j] = fano_fit(
            y[f], (c0[f], dbar, bbar), w, q, box, max_iter, tol)
        out[j] = (c, w, d, b)
    return out, iters, status, chi2
