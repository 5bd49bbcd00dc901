"""FP64 forward/backward of the learned warm-start network, loss and Adam.

Test infrastructure only (see the package docstring).

The learned warm start maps a normalised tooth vector (K = 220 amplitudes) to
standardised start parameters (c, w, d, b) of the Lorentzian fit:

    h1 = W1 x + b1,  a1 = GELU(h1)          (220 -> 256)
    h2 = W2 a1 + b2, a2 = GELU(h2)          (256 -> 256)
    out = W3 a2 + b3                        (256 -> 4)

GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 (exact erf), so
GELU'(z) = Phi(z) + z phi(z).  Loss: weighted mean squared error over the
batch and the four outputs, L = sum_s m_s sum_j (out_sj - t_sj)^2 / (4 sum_s m_s)
with per-sample weights m_s (1 for kept samples, 0 for dropped ones).  Adam
(Kingma & Ba 2015) with bias correction.

Mixed precision of the GPU kernels: every operand of a matrix product is
rounded to bfloat16 (round to nearest even) and the products are summed in
full precision; bias additions, GELU, the loss and Adam stay in full
precision.  `bf16_ops=True` emulates exactly those rounding points (sums in FP64
here); `bf16_ops=False` is plain FP64 (used to pin the backward pass against
finite differences).

Flat parameter layout: W1[256][220], b1[256], W2[256][256], b2[256],
W3[4][256], b3[4] (123 396 values).
"""

import math

import numpy as np
from scipy.special import erf as _erf

IN, HID, OUT = 220, 256, 4
SHAPES = [("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
          ("W3", (OUT, HID)), ("b3", (OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16(a):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = p[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    cdf = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    pdf = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return cdf + z * pdf


def forward(x, params, bf16_ops=True):
    """x [B, 220] -> out [B, 4] and the cache for backward."""
    r = bf16 if bf16_ops else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(params)
    x = np.asarray(x, dtype=np.float64)
    xq = r(x)
    h1 = xq @ r(p["W1"]).T + p["b1"]
    a1 = gelu(h1)
    a1q = r(a1)
    h2 = a1q @ r(p["W2"]).T + p["b2"]
    a2 = gelu(h2)
    a2q = r(a2)
    out = a2q @ r(p["W3"]).T + p["b3"]
    cache = {"xq": xq, "h1": h1, "a1q": a1q, "h2": h2, "a2q": a2q, "p": p, "r": r}
    return out, cache


def loss_and_dout(out, target, weight=None):
    out = np.asarray(out, dtype=np.float64)
    t = np.asarray(target, dtype=np.float64)
    w = np.ones(out.shape[0]) if weight is None else np.asarray(weight, dtype=np.float64)
    denom = 4.0 * w.sum()
    diff = out - t
    loss = float(np.sum(w[:, None] * diff * diff) / denom)
    dout = 2.0 * w[:, None] * diff / denom
    return loss, dout


def backward(cache, dout):
    r, p = cache["r"], cache["p"]
    g = {}
    d3 = r(dout)
    g["W3"] = d3.T @ cache["a2q"]
    g["b3"] = dout.sum(axis=0)
    da2 = d3 @ r(p["W3"])
    dh2 = da2 * gelu_grad(cache["h2"])
    dh2q = r(dh2)
    g["W2"] = dh2q.T @ cache["a1q"]
    g["b2"] = dh2.sum(axis=0)
    da1 = dh2q @ r(p["W2"])
    dh1 = da1 * gelu_grad(cache["h1"])
    dh1q = r(dh1)
    g["W1"] = dh1q.T @ cache["xq"]
    g["b1"] = dh1.sum(axis=0)
    return pack(g)


def loss_and_grads(x, target, params, weight=None, bf16_ops=True):
    out, cache = forward(x, params, bf16_ops)
    loss, dout = loss_and_dout(out, target, weight)
    return loss, backward(cache, dout)


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns (params, m, v)."""
    g = np.asarray(grads, dtype=np.float64)
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def resample_to_input(y, k_in=IN):
    """Linear resampling of a K-tooth vector onto 220 points over the same
    normalised axis (used when K != 220)."""
    y = np.asarray(y, dtype=np.float64)
    k = y.shape[-1]
    if k == k_in:
        return y
    pos = np.arange(k_in) * (k - 1) / (k_in - 1)
    lo = np.clip(np.floor(pos).astype(int), 0, k - 1)
    hi = np.clip(lo + 1, 0, k - 1)
    fr = pos - lo
    return y[..., lo] * (1.0 - fr) + y[..., hi] * fr
