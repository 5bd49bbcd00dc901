"""Levenberg-Marquardt fit of the Lorentzian cavity dip (FP64).

Test infrastructure only (see the package docstring).

Paper, Data Capture and Processing: every normalised spectrum is fitted by a
Levenberg-Marquardt least-squares routine, at most 20 iterations, tolerance
1e-6; the centre of the cavity resonance is the quantity of interest (a shift
of the resonance is a change of cavity length, i.e. proof-mass displacement,
Experimental Setup).  The paper fits a 5-parameter Fano shape; the path built
here fits the 4-parameter Lorentzian dip

    f(x; c, w, d, b) = b (1 - d / (1 + u^2)),   u = 2 (x - c) / w,

over the tooth index x = 0..K-1 (c = centre and w = FWHM in teeth, d = depth,
b = baseline), by unweighted least squares chi2 = sum (y - f)^2.

Readings for the iteration schedule (the paper names only the cap and the
tolerance):
* damped normal equations (A + lam diag(A)) delta = g, A = J^T J, g = J^T r,
  r = y - f, solved by Cholesky; lam starts at 1e-3, is divided by 10 after an
  accepted step and multiplied by 10 after a rejected one;
* one iteration = one solve plus the evaluation of the trial point, accepted or
  not; at most `max_iter` of them;
* a trial point is rejected when it is not finite, has w <= 0, or does not
  lower chi2 (chi2_new <= chi2_old is accepted);
* converged (status 0) when an accepted step lowers chi2 by at most
  tol * chi2_old, or chi2 reaches 1e-30;
* a failed Cholesky (A + lam diag(A) not positive definite) stops the fit with
  status 2; running out of iterations gives status 1.
The returned parameters are always the last accepted point.
"""

import numpy as np

STATUS_CONVERGED = 0
STATUS_MAX_ITER = 1
STATUS_SINGULAR = 2


def lorentzian(x, p):
    c, w, d, b = (float(v) for v in p)
    u = 2.0 * (np.asarray(x, dtype=np.float64) - c) / w
    return b * (1.0 - d / (1.0 + u * u))


def lorentzian_jacobian(x, p):
    """Analytic partial derivatives [K, 4] in the order (c, w, d, b).

    With u = 2 (x - c)/w and D = 1 + u^2:
      df/dc = -4 b d u / (w D^2),  df/dw = -2 b d u^2 / (w D^2),
      df/dd = -b / D,              df/db = 1 - d / D.
    """
    c, w, d, b = (float(v) for v in p)
    x = np.asarray(x, dtype=np.float64)
    u = 2.0 * (x - c) / w
    den = 1.0 + u * u
    jac = np.empty((x.shape[0], 4))
    jac[:, 0] = -4.0 * b * d * u / (w * den * den)
    jac[:, 1] = -2.0 * b * d * u * u / (w * den * den)
    jac[:, 2] = -b / den
    jac[:, 3] = 1.0 - d / den
    return jac


def chi2_at(y, p) -> float:
    """chi2 = sum_i (y_i - f(i; p))^2 evaluated in FP64."""
    y = np.asarray(y, dtype=np.float64)
    r = y - lorentzian(np.arange(y.shape[0]), p)
    return float(r @ r)


def _cholesky_solve(a, g):
    try:
        low = np.linalg.cholesky(a)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(low)):
        return None
    z = np.linalg.solve(low, g)
    return np.linalg.solve(low.T, z)


def lm_fit(y, p0, max_iter: int = 20, tol: float = 1e-6, lam0: float = 1e-3, trace=None):
    """Fit one spectrum.  Returns (params[4], iterations, status, chi2).

    If `trace` is a list, one dict per iteration is appended to it with the
    point the step started from, the damping used, the step and whether the
    trial point was accepted.
    """
    y = np.asarray(y, dtype=np.float64)
    x = np.arange(y.shape[0], dtype=np.float64)
    p = np.asarray(p0, dtype=np.float64).copy()

    r = y - lorentzian(x, p)
    chi2 = float(r @ r)
    jac = lorentzian_jacobian(x, p)
    a = jac.T @ jac
    g = jac.T @ r
    lam = lam0
    status = STATUS_MAX_ITER
    it = 0
    if not np.isfinite(chi2):
        return p, 0, STATUS_SINGULAR, chi2
    if chi2 <= 1e-30:
        return p, 0, STATUS_CONVERGED, chi2
    while it < max_iter:
        it += 1
        damped = a + lam * np.diag(np.diag(a))
        delta = _cholesky_solve(damped, g)
        if delta is None:
            status = STATUS_SINGULAR
            break
        trial = p + delta
        ok = bool(np.all(np.isfinite(trial))) and trial[1] > 0.0
        if ok:
            r_t = y - lorentzian(x, trial)
            chi2_t = float(r_t @ r_t)
            ok = np.isfinite(chi2_t) and chi2_t <= chi2
        if trace is not None:
            trace.append({"p": p.copy(), "lam": lam, "delta": delta.copy(), "accepted": bool(ok)})
        if not ok:
            lam *= 10.0
            continue
        drop = chi2 - chi2_t
        old = chi2
        p = trial
        chi2 = chi2_t
        jac = lorentzian_jacobian(x, p)
        a = jac.T @ jac
        g = jac.T @ r_t
        lam /= 10.0
        if drop <= tol * old or chi2 <= 1e-30:
            status = STATUS_CONVERGED
            break
    return p, it, status, chi2


def lm_fit_batch(y, p0, max_iter: int = 20, tol: float = 1e-6):
    """Fit every row of y [F, K] from p0 [F, 4] (plain loop over frames)."""
    y = np.asarray(y, dtype=np.float64)
    p0 = np.asarray(p0, dtype=np.float64)
    f_count = y.shape[0]
    params = np.empty((f_count, 4))
    iters = np.empty(f_count, dtype=np.int32)
    status = np.empty(f_count, dtype=np.int32)
    chi2 = np.empty(f_count)
    for f in range(f_count):
        params[f], iters[f], status[f], chi2[f] = lm_fit(y[f], p0[f], max_iter, tol)
    return params, iters, status, chi2
