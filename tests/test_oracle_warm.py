"""Pins of the oracle's learned warm start (network start point, polish and
cold-start fallback), each against a closed form rather than the oracle's own
arithmetic:

* a network whose weights are zero outputs its last bias, so the start point
  is that bias mapped through the output mean and spread and, for K != 220,
  scaled by (K - 1) / 219 in centre and width;
* a network that routes one input through both hidden layers (weights 16,
  1, 1/16 on positive inputs, where GELU is the identity to far below one
  bfloat16 step) outputs the resampled spectrum's value at that input, which
  for a linear ramp is known in closed form;
* spectra built as a noiseless Lorentzian plus a residual orthogonal to the
  model's Jacobian at the true point have a known minimum chi2, which puts a
  frame exactly on either side of the fallback threshold
  chi2 = 4 sigma^2 (K - 4) (RMS residual = 2 sigma).
"""

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from oracle.pipeline import network_start, warm_fit


def _dip(k, c, w, d, b):
    x = np.arange(k, dtype=np.float64)
    return b * (1.0 - d / (1.0 + (2.0 * (x - c) / w) ** 2))


def _bias_network(z):
    p = np.zeros(mlp.N_PARAMS)
    p[-4:] = z
    return p


@pytest.mark.parametrize("k", [220, 100, 440])
def test_zero_network_start_is_output_bias(k):
    z = np.array([0.25, -0.5, 1.5, -2.0])
    mean = np.array([100.0, 9.0, 0.4, 1.0])
    std = np.array([30.0, 4.0, 0.2, 0.05])
    y = np.random.default_rng(k).random((5, k)) + 0.5
    p0 = network_start(y, _bias_network(z), mean, std)
    want = z * std + mean
    want[:2] *= (k - 1) / 219.0
    assert np.allclose(p0, np.broadcast_to(want, p0.shape), rtol=0, atol=1e-12)


@pytest.mark.parametrize("k,j", [(100, 0), (100, 37), (100, 219), (220, 111), (440, 150)])
def test_routing_network_sees_resampled_input(k, j):
    p = mlp.unpack(np.zeros(mlp.N_PARAMS))
    p["W1"][0, j] = 16.0
    p["W2"][0, 0] = 1.0
    p["W3"][0, 0] = 1.0 / 16.0
    ramp = 0.5 + np.arange(k) / 64.0           # exact in float32
    y = np.tile(ramp, (3, 1))
    p0 = network_start(y, mlp.pack(p), np.zeros(4), np.ones(4))
    # linear resampling of a ramp onto 220 points over the same axis is the
    # ramp at position j (k - 1) / 219; the network rounds it to bfloat16
    val = 0.5 + (j * (k - 1) / 219.0) / 64.0
    val_bf16 = torch.tensor(val, dtype=torch.float32).to(torch.bfloat16).double().item()
    want_c = val_bf16 * (k - 1) / 219.0
    assert np.allclose(p0[:, 0], want_c, rtol=0, atol=1e-12)
    assert np.allclose(p0[:, 1], 0.0, atol=1e-12)
    assert np.allclose(p0[:, 2:], 0.0, atol=1e-12)


def _orthogonal_residual_spectrum(k, truth, s_target, seed):
    """Noiseless dip plus a residual e with |e|^2 = s_target that is
    orthogonal to the four columns of the model's Jacobian at `truth`
    (Jacobian by central differences of the test's own model)."""
    c, w, d, b = truth
    base = _dip(k, c, w, d, b)
    jac = np.empty((k, 4))
    for j in range(4):
        h = 1e-6 * max(1.0, abs(truth[j]))
        tp, tm = list(truth), list(truth)
        tp[j] += h
        tm[j] -= h
        jac[:, j] = (_dip(k, *tp) - _dip(k, *tm)) / (2 * h)
    e = np.random.default_rng(seed).standard_normal(k)
    q, _ = np.linalg.qr(jac)
    e -= q @ (q.T @ e)
    e *= np.sqrt(s_target / (e @ e))
    return base + e


@pytest.mark.parametrize("k", [220, 100])
def test_fallback_threshold_straddles_exactly(k):
    truth = (0.45 * k, 9.0, 0.6, 1.0)
    sigma = 0.01
    thr2 = 4.0 * sigma ** 2 * (k - 4)
    below = _orthogonal_residual_spectrum(k, truth, thr2 * (1 - 1e-6), 1)
    above = _orthogonal_residual_spectrum(k, truth, thr2 * (1 + 1e-6), 2)
    y = np.vstack([below, above])
    p0 = np.array([truth, truth], dtype=np.float64)
    params, iters, status, chi2, fell = warm_fit(y, p0, sigma, polish_iter=2)
    # the start point is already the minimum: the polish keeps it
    assert not fell[0] and status[0] in (0, 1) and iters[0] <= 2
    assert np.allclose(params[0], truth, rtol=0, atol=1e-9)
    assert abs(chi2[0] / (thr2 * (1 - 1e-6)) - 1) < 1e-9
    # just above the threshold: refitted from the cold start, status 3, and
    # the iteration count reported is the refit's
    assert fell[1] and status[1] == 3
    cold = oracle.initial_guess(y)
    _, it_cold, _, c2_cold = oracle.lm_fit(y[1], cold[1], 20, 1e-6)
    assert iters[1] == it_cold and chi2[1] == c2_cold


def test_non_finite_polish_falls_back():
    k = 220
    y = _dip(k, 100.0, 9.0, 0.6, 1.0)[None, :] + 1e-3
    p0 = np.array([[100.0, 0.0, 0.6, 1.0]])      # zero width: the model is not finite
    params, iters, status, chi2, fell = warm_fit(y, p0, 0.01)
    assert fell[0] and status[0] == 3 and np.isfinite(chi2[0])
    assert abs(params[0, 0] - 100.0) < 0.05


def test_polish_from_exact_start_on_noiseless_spectra():
    """From the true point of a noiseless spectrum the polish stops at once
    (chi2 at rounding level) and no frame falls back."""
    k = 100
    truths = [(30.0, 6.0, 0.5, 1.0), (61.5, 12.0, 0.8, 0.97), (5.25, 4.0, 0.3, 1.02)]
    y = np.vstack([_dip(k, *t) for t in truths])
    params, iters, status, chi2, fell = warm_fit(y, np.array(truths), 1e-3)
    assert not fell.any() and np.all(status == 0) and np.all(iters <= 1)
    assert np.allclose(params, truths, rtol=0, atol=1e-9)


def test_row_sampled_warm_fit_equals_full_batch_rows():
    k = 100
    rng = np.random.default_rng(3)
    truths = [(20.0 + 3 * i, 8.0, 0.6, 1.0) for i in range(12)]
    y = np.vstack([_dip(k, *t) for t in truths]) + 0.01 * rng.standard_normal((12, k))
    p0 = np.array(truths) + [0.3, 0.5, 0.02, 0.0]
    full = warm_fit(y, p0, 0.005)
    rows = np.array([0, 1, 5, 6, 9])
    part = warm_fit(y, p0[rows], 0.005, rows=rows)
    for a, b in zip(full, part):
        assert np.array_equal(a[rows], b)
    assert full[4].any() and not full[4].all()      # both branches exercised
