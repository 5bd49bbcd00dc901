"""Pins of the oracle's warm-start network: finite differences, GELU closed
forms, bfloat16 rounding and Adam against torch's CPU implementations."""

import numpy as np
import pytest
import torch

from oracle import mlp


def _params(seed, scale=0.1):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(mlp.N_PARAMS) * scale


def test_param_count():
    assert mlp.N_PARAMS == 123396
    p = _params(0)
    assert np.array_equal(mlp.pack(mlp.unpack(p)), p)


def test_gelu_closed_forms():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5)
    z = np.linspace(-6, 6, 101)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    assert np.max(np.abs(mlp.gelu(z) - ref)) <= 1e-12
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.gelu_grad(z))) <= 1e-8
    assert mlp.gelu(np.array([40.0]))[0] == pytest.approx(40.0)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    a = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 0.0, 65504.0]])
    want = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(a), want)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = _params(3, 0.05)
    x = rng.random((6, mlp.IN))
    t = rng.standard_normal((6, mlp.OUT))
    w = np.array([1, 1, 0, 1, 1, 1], dtype=np.float64)
    loss, g = mlp.loss_and_grads(x, t, p, w, bf16_ops=False)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, mlp.N_PARAMS - 5, 56320, 56320 + 256]])
    for i in idx:
        h = 1e-5
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp.loss_and_grads(x, t, pp, w, False)[0] - mlp.loss_and_grads(x, t, pm, w, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_fp64_forward_matches_torch():
    rng = np.random.default_rng(4)
    p = _params(5)
    x = rng.random((9, mlp.IN))
    out, _ = mlp.forward(x, p, bf16_ops=False)
    d = {k: torch.from_numpy(v) for k, v in mlp.unpack(p).items()}
    h = torch.nn.functional.gelu(torch.from_numpy(x) @ d["W1"].T + d["b1"])
    h = torch.nn.functional.gelu(h @ d["W2"].T + d["b2"])
    ref = (h @ d["W3"].T + d["b3"]).numpy()
    assert np.max(np.abs(out - ref)) <= 1e-12


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    p0 = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p = p0.copy()
    for step in range(1, 6):
        g = rng.standard_normal(50)
        p, m, v = mlp.adam_step(p, g, m, v, step)
        opt.zero_grad()
        tp.grad = torch.from_numpy(g)
        opt.step()
    assert np.max(np.abs(p - tp.detach().numpy())) <= 1e-12
    # first step moves every parameter by lr in the direction of -sign(g)
    g = rng.standard_normal(50)
    p1, _, _ = mlp.adam_step(p0, g, np.zeros(50), np.zeros(50), 1)
    assert np.allclose(p1 - p0, -1e-3 * np.sign(g), rtol=1e-6)


def test_resample_identity_and_endpoints():
    y = np.random.default_rng(7).random((3, 100))
    r = mlp.resample_to_input(y)
    assert r.shape == (3, 220)
    assert np.allclose(r[:, 0], y[:, 0]) and np.allclose(r[:, -1], y[:, -1])
    z = np.random.default_rng(8).random((2, 220))
    assert np.array_equal(mlp.resample_to_input(z), z)
    lin = np.linspace(0, 1, 64)[None, :]
    assert np.allclose(mlp.resample_to_input(lin), np.linspace(0, 1, 220)[None, :])
