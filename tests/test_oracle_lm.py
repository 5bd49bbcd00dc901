"""Pins of the oracle's Levenberg-Marquardt Lorentzian fit."""

import numpy as np
import pytest
from scipy.optimize import least_squares

import oracle
import synth


def test_jacobian_matches_finite_differences():
    rng = np.random.default_rng(2)
    x = np.arange(220, dtype=np.float64)
    for _ in range(20):
        p = np.array([rng.uniform(50, 170), rng.uniform(3, 20), rng.uniform(0.1, 0.9),
                      rng.uniform(0.8, 1.2)])
        jac = oracle.lorentzian_jacobian(x, p)
        for j in range(4):
            h = 1e-6 * max(1.0, abs(p[j]))
            pp, pm = p.copy(), p.copy()
            pp[j] += h
            pm[j] -= h
            fd = (oracle.lorentzian(x, pp) - oracle.lorentzian(x, pm)) / (2 * h)
            assert np.max(np.abs(fd - jac[:, j])) <= 1e-6 * max(1.0, np.abs(jac[:, j]).max())


@pytest.mark.parametrize("k,centre,width", [(100, (40, 60), (8, 8)), (220, (90, 130), (4, 16)),
                                            (220, (70, 150), (3, 20)), (64, (25, 40), (4, 16)),
                                            (440, (200, 240), (4, 16))])
def test_exact_recovery_noiseless(k, centre, width):
    y, truth, _ = synth.make_lorentzian_spectra(k, 40, seed=k, centre=centre, width=width,
                                                depth=(0.1, 0.9), baseline=(0.9, 1.1))
    rng = np.random.default_rng(k + 1)
    for f in range(y.shape[0]):
        p0 = truth[f] * np.array([1, 1.2, 1, 1]) + np.array([rng.uniform(-1.5, 1.5), 0,
                                                             rng.uniform(-0.05, 0.05), 0.02])
        p, it, st, chi2 = oracle.lm_fit(y[f], p0, max_iter=40)
        assert st == 0, (f, it, chi2)
        assert np.max(np.abs(p - truth[f]) / np.abs(truth[f])) <= 1e-9


def test_first_order_optimality_and_scipy_minpack():
    """On noisy spectra the fully converged fit has J^T r ~ 0 and agrees with
    MINPACK's Levenberg-Marquardt (scipy, FP64) to 1e-8 FWHM in the centre."""
    k = 220
    y, truth, _ = synth.make_lorentzian_spectra(k, 30, seed=9, centre=(90, 130), width=(4, 16),
                                                depth=(0.6, 0.6), sigma=(0.003, 0.03))
    x = np.arange(k, dtype=np.float64)
    for f in range(y.shape[0]):
        p, it, st, _ = oracle.lm_fit(y[f], truth[f] + [0.7, 1.0, -0.05, 0.01], max_iter=200,
                                     tol=1e-14)
        assert st == 0
        r = y[f] - oracle.lorentzian(x, p)
        g = oracle.lorentzian_jacobian(x, p).T @ r
        assert np.max(np.abs(g)) <= 1e-7 * np.linalg.norm(y[f])
        ls = least_squares(lambda q: y[f] - oracle.lorentzian(x, q), truth[f], method="lm",
                           xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=10000)
        assert abs(ls.x[0] - p[0]) <= 1e-8 * p[1]


def test_centre_spread_matches_cramer_rao():
    """Over many noise draws the spread of fitted centres equals the Cramer-Rao
    bound sigma * sqrt([(J^T J)^-1]_cc) within 10 %."""
    k, n = 100, 1500
    p_true = np.array([49.5, 8.0, 0.6, 1.0])
    sigma = 0.01
    x = np.arange(k, dtype=np.float64)
    clean = oracle.lorentzian(x, p_true)
    rng = np.random.default_rng(123)
    cs = np.empty(n)
    for j in range(n):
        y = clean + sigma * rng.standard_normal(k)
        p, _, st, _ = oracle.lm_fit(y, p_true + [1.0, 1.0, 0.05, 0.0])
        assert st == 0
        cs[j] = p[0]
    jac = oracle.lorentzian_jacobian(x, p_true)
    crlb = sigma * np.sqrt(np.linalg.inv(jac.T @ jac)[0, 0])
    assert 0.9 < np.std(cs) / crlb < 1.1
    assert abs(np.mean(cs) - p_true[0]) < 4 * crlb / np.sqrt(n)


def test_schedule_status_codes():
    k = 50
    x = np.arange(k, dtype=np.float64)
    y = oracle.lorentzian(x, [25.0, 6.0, 0.5, 1.0]) + 0.01 * np.sin(x)
    # a single iteration from a distant start cannot meet the tolerance
    p, it, st, _ = oracle.lm_fit(y, [20.0, 9.0, 0.3, 0.9], max_iter=1)
    assert it == 1 and st == 1
    # zero baseline: the columns for c, w, d vanish -> singular normal equations
    p, it, st, _ = oracle.lm_fit(y, [25.0, 6.0, 0.5, 0.0])
    assert st == 2 and it == 1
    # iteration count never exceeds the cap
    rng = np.random.default_rng(0)
    for _ in range(20):
        yy = y + 0.2 * rng.standard_normal(k)
        _, it, st, _ = oracle.lm_fit(yy, [10.0, 3.0, 0.9, 1.2])
        assert 1 <= it <= 20 and st in (0, 1)


def test_chi2_never_increases():
    k = 220
    y, truth, _ = synth.make_lorentzian_spectra(k, 20, seed=4, centre=(90, 130), width=(4, 16),
                                                depth=(0.6, 0.6), sigma=(0.01, 0.1))
    for f in range(y.shape[0]):
        p0 = truth[f] + [5.0, 3.0, -0.2, 0.05]
        c0 = oracle.chi2_at(y[f], p0)
        p, it, st, chi2 = oracle.lm_fit(y[f], p0)
        assert chi2 <= c0
        assert chi2 == pytest.approx(oracle.chi2_at(y[f], p), rel=1e-12)


def test_steps_solve_damped_least_squares_and_schedule():
    """Every step minimises |J delta - r|^2 + lam delta^T diag(J^T J) delta, checked
    through an independent route (SVD least squares of the augmented system
    [J; sqrt(lam D)] delta = [r; 0]); the damping starts at 1e-3 and moves by a
    factor 10 down after an accepted and up after a rejected step."""
    k = 120
    x = np.arange(k, dtype=np.float64)
    rng = np.random.default_rng(77)
    saw_reject = False
    for trial in range(12):
        y = oracle.lorentzian(x, [60.0, 7.0, 0.5, 1.0]) + 0.05 * rng.standard_normal(k)
        tr = []
        oracle.lm_fit(y, [60.0 + rng.uniform(-12, 12), 14.0, 0.2, 0.9], trace=tr)
        assert tr[0]["lam"] == 1e-3
        for a, b in zip(tr, tr[1:]):
            assert b["lam"] == pytest.approx(a["lam"] / 10 if a["accepted"] else a["lam"] * 10,
                                             rel=1e-12)
            saw_reject |= not a["accepted"]
        for st in tr:
            jac = oracle.lorentzian_jacobian(x, st["p"])
            r = y - oracle.lorentzian(x, st["p"])
            dmat = np.diag(np.sqrt(st["lam"] * np.sum(jac * jac, axis=0)))
            aug = np.vstack([jac, dmat])
            rhs = np.concatenate([r, np.zeros(4)])
            want = np.linalg.lstsq(aug, rhs, rcond=None)[0]
            assert np.allclose(st["delta"], want, rtol=1e-7, atol=1e-10 * np.abs(want).max())
    assert saw_reject
