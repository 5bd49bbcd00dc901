"""Pins of the oracle's Fano fit (the paper's own lineshape: centre free,
extent and scale boxed to +-10 % of batch averages, width and asymmetry
fixed), against things other than the oracle itself:
* the q -> infinity limit is the plain path's Lorentzian dip, and a fit in
  that limit agrees with the Lorentzian LM on noiseless spectra;
* the analytic Jacobian matches central finite differences;
* noiseless Fano spectra are recovered exactly from perturbed starts;
* fully converged fits agree with scipy's bounded trust-region least squares
  (method 'trf'), including fits that end on a bound of the box;
* the box is +-10 % of the pre-calculated averages."""

import numpy as np
import pytest
from scipy.optimize import least_squares

import oracle
from oracle.fano import fano, fano_box, fano_fit, fano_jacobian


def _spectrum(k, c, w, d, b, q, sigma=0.0, seed=0):
    x = np.arange(k, dtype=np.float64)
    u = 2.0 * (x - c) / w
    y = b * (1.0 - d * (1.0 + u / q) ** 2 / (1.0 + u * u))
    if sigma:
        y = y + sigma * np.random.default_rng(seed).standard_normal(k)
    return y


def test_infinite_asymmetry_is_the_lorentzian():
    x = np.arange(220.0)
    p = (101.3, 8.0, 0.6, 1.02)
    assert np.max(np.abs(fano(x, *p, q=1e12) - oracle.lorentzian(x, p))) < 1e-10
    # finite q tilts the dip: deepest point at u = 1/q with depth d (1 + 1/q^2)
    q = 3.0
    xs = np.linspace(90, 110, 200001)
    f = fano(xs, 101.3, 8.0, 0.6, 1.0, q)
    i = np.argmin(f)
    assert abs(xs[i] - (101.3 + 8.0 / (2 * q))) < 1e-3
    assert abs(f[i] - (1.0 - 0.6 * (1 + 1 / q ** 2))) < 1e-9


@pytest.mark.parametrize("q", [2.5, -4.0, 30.0])
def test_jacobian_matches_finite_differences(q):
    x = np.arange(120.0)
    c, w, d, b = 57.4, 9.5, 0.55, 0.97
    jac = fano_jacobian(x, c, w, d, b, q)
    for j, (name, h) in enumerate((("c", 1e-6), ("d", 1e-7), ("b", 1e-7))):
        hi = dict(c=c, d=d, b=b)
        lo = dict(c=c, d=d, b=b)
        hi[name] += h
        lo[name] -= h
        fd = (fano(x, hi["c"], w, hi["d"], hi["b"], q) - fano(x, lo["c"], w, lo["d"], lo["b"], q)) / (2 * h)
        assert np.max(np.abs(fd - jac[:, j])) < 1e-7 * max(1.0, np.max(np.abs(fd)))


@pytest.mark.parametrize("q", [3.0, -5.0, 1e9])
def test_noiseless_recovery(q):
    k, w = 220, 8.03
    truth = (108.7, 0.6, 1.03)
    y = _spectrum(k, truth[0], w, truth[1], truth[2], q)
    box = np.array([[0.5, 0.7], [0.95, 1.1]])
    for start in ((104.0, 0.55, 1.0), (113.0, 0.68, 1.08), (108.0, 0.6, 1.03)):
        (c, d, b), it, st, chi2 = fano_fit(y, start, w, q, box)
        assert st == 0 and it <= 20
        assert np.allclose((c, d, b), truth, rtol=0, atol=1e-8), (start, c, d, b)


def test_lorentzian_limit_agrees_with_plain_fit():
    k = 220
    y = _spectrum(k, 99.2, 12.0, 0.45, 0.98, 1e12)
    (c, d, b), _, st, _ = fano_fit(y, (96.0, 0.4, 1.0), 12.0, 1e12,
                                   np.array([[0.3, 0.6], [0.9, 1.1]]))
    p, _, st2, _ = oracle.lm_fit(y, (96.0, 12.0, 0.4, 1.0))
    assert st == 0 and st2 == 0
    assert np.allclose((c, d, b), (p[0], p[2], p[3]), atol=1e-8)


def _scipy_fit(y, start, w, q, box):
    x = np.arange(y.shape[0], dtype=np.float64)
    lo = [-np.inf, box[0][0], box[1][0]]
    hi = [np.inf, box[0][1], box[1][1]]
    st = np.clip(start, lo, hi)
    res = least_squares(lambda p: fano(x, p[0], w, p[1], p[2], q) - y, st, method="trf",
                        bounds=(lo, hi), xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=10000)
    return res.x


@pytest.mark.parametrize("case", range(6))
def test_converged_fit_agrees_with_scipy_bounded(case):
    rng = np.random.default_rng(case)
    k, w, q = 220, 8.03, 4.0
    c = 100 + 20 * rng.random()
    d = 0.6
    b = 1.0 + 0.3 * (case % 3 - 1) * (case >= 3)     # cases 3 and 5 put the truth outside the box
    y = _spectrum(k, c, w, d, b, q, sigma=0.01, seed=case)
    box = np.array([[0.54, 0.66], [0.9, 1.1]])
    start = (c + 2.0, 0.58, 1.0)
    (fc, fd, fb), it, st, chi2 = fano_fit(y, start, w, q, box, max_iter=200, tol=1e-14)
    ref = _scipy_fit(y, start, w, q, box)
    assert np.allclose((fc, fd, fb), ref, rtol=0, atol=1e-6), ((fc, fd, fb), ref)
    if case in (3, 5):
        bound = 1.1 if b > 1 else 0.9
        assert fb == bound and abs(ref[2] - bound) < 1e-9


def test_projection_keeps_the_box():
    k, w, q = 150, 8.0, 4.0
    y = _spectrum(k, 70.0, w, 0.9, 1.4, q, sigma=0.002, seed=3)
    box = np.array([[0.5, 0.6], [0.9, 1.1]])
    (c, d, b), it, st, chi2 = fano_fit(y, (72.0, 0.55, 1.0), w, q, box)
    assert 0.5 <= d <= 0.6 and b == 1.1   # the scale is held on its upper bound
    assert abs(c - 70.0) < 1.5           # 20 iterations do not reach the optimum here
    (c, d, b), it, st, chi2 = fano_fit(y, (72.0, 0.55, 1.0), w, q, box, max_iter=200, tol=1e-14)
    ref = _scipy_fit(y, (72.0, 0.55, 1.0), w, q, box)
    assert st == 0 and np.allclose((c, d, b), ref, atol=1e-6) and b == 1.1


def test_box_is_ten_percent_of_the_averages():
    assert np.allclose(fano_box(0.6, 1.02), [[0.54, 0.66], [0.918, 1.122]])


def test_fano_stream_end_to_end_recovers_truth():
    """The oracle's whole Fano path on the paper-rate Fano stream: centres
    within the noise of the truth, extent and scale inside the box."""
    import synth
    from oracle.pipeline import process_batch_fano
    spec = synth.spec_fano()
    bt = synth.make_batch(spec, 256, seed=31)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins)
    out = process_batch_fano(bt.frames, spec.bins, ref, 8.03, 4.0, 0.6, 1.0)
    box = out["box"]
    p = out["params"]
    assert np.all((p[:, 2] >= box[0, 0]) & (p[:, 2] <= box[0, 1]))
    assert np.all((p[:, 3] >= box[1, 0]) & (p[:, 3] <= box[1, 1]))
    assert np.mean(out["status"] == 0) > 0.95
    err = np.abs(p[:, 0] - bt.centre) / 8.03
    assert np.median(err) < 0.01
    assert 2.0 <= np.mean(out["iters"]) <= 8.0


def test_paper_geometry_int8_stream_end_to_end():
    """The paper's own configuration (8-bit 2200-sample frames, teeth
    |51 + 10 n| MHz, Fano dip): the oracle's whole path recovers the centre
    within the noise of the 8-bit stream."""
    import synth
    from oracle.pipeline import process_batch_fano
    spec = synth.spec_paper8()
    bt = synth.make_batch(spec, 192, seed=8)
    ref = oracle.reference_spectrum(bt.ref_frames, spec.bins)
    out = process_batch_fano(bt.frames, spec.bins, ref, 8.03, 4.0, 0.6, 1.0)
    err = np.abs(out["params"][:, 0] - bt.centre) / 8.03
    assert np.mean(out["status"] == 0) > 0.95
    assert np.median(err) < 0.02
