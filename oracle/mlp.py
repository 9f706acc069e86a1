"""FP64 oracle of the learned sun-visibility surrogate (a small MLP).

TEST INFRASTRUCTURE ONLY (tests, smoke, the benchmark's CPU-baseline leg).  The
surrogate is not in the paper: it is specified from first principles as a stand-in for
the geometric shadow pass (Sec. 3.1 image formation, V; Sec. 3.3 sun camera), and the
geometric pass stays both its training-label source and its fallback.

Network (all choices stated here, none taken from the paper):
  input   p_hat = fl32(fl32(p - centre) * inv_half)       (FP32, per coordinate)
          features[32c + 2k]     = sin(pi 2^k p_hat_c)      c = 0..2, k = 0..15
          features[32c + 2k + 1] = cos(pi 2^k p_hat_c)
          features[96..99]       = cos phi, sin phi, sin theta, cos theta
          features[100..127]     = 0
  layers  h1 = relu(W1 f + b1), W1 [64,128]
          h2 = relu(W2 h1 + b2), W2 [64,64]
          h3 = relu(W3 h2 + b3), W3 [64,64]
          logit = w4 . h3 + b4,  p = sigmoid(logit)
  params  one FP32 vector [W1, b1, W2, b2, W3, b3, w4, b4] (16641 floats)
  BF16    (when bf16=True) features, weights W1..W3 and w4, and the hidden activations
          h1..h3 are rounded to bfloat16 (round to nearest even) before they enter a
          product; sums are exact (FP64 here).  In the backward the pre-activation
          gradients da3, da2, da1 are rounded to bfloat16 before they enter a product
          (dW, db and the propagated dh all use the rounded values).
The exact sin/cos range reduction: x = 2^k p_hat is exact, r = x - 2 rint(x/2) is exact,
and sin(pi x) = sin(pi r).
"""
from __future__ import annotations

import numpy as np

N_FREQ = 16
IN = 128
WIDTH = 64
SIZES = dict(W1=(WIDTH, IN), b1=(WIDTH,), W2=(WIDTH, WIDTH), b2=(WIDTH,), W3=(WIDTH, WIDTH),
             b3=(WIDTH,), w4=(WIDTH,), b4=(1,))
N_PARAMS = sum(int(np.prod(s)) for s in SIZES.values())


def unpack(w):
    out, o = {}, 0
    for k, s in SIZES.items():
        n = int(np.prod(s))
        out[k] = np.asarray(w[o:o + n], np.float64).reshape(s)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[k], np.float64).reshape(-1) for k in SIZES])


def bf16(x):
    """Round to bfloat16 (round to nearest even), via FP32, returned as float64."""
    f = np.asarray(x, np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def normalise(pts, centre, inv_half):
    p = np.asarray(pts, np.float32)
    c = np.asarray(centre, np.float32)
    s = np.float32(inv_half)
    return ((p - c).astype(np.float32) * s).astype(np.float32)


def features(pts, sun, centre, inv_half, rounding=True):
    ph = normalise(pts, centre, inv_half).astype(np.float64)         # [M,3], exact FP32 values
    M = ph.shape[0]
    f = np.zeros((M, IN))
    for c in range(3):
        for k in range(N_FREQ):
            x = ph[:, c] * (2.0 ** k)
            r = x - 2.0 * np.rint(x / 2.0)
            f[:, 32 * c + 2 * k] = np.sin(np.pi * r)
            f[:, 32 * c + 2 * k + 1] = np.cos(np.pi * r)
    phi = np.asarray(sun, np.float32)[:, 0].astype(np.float64)
    th = np.asarray(sun, np.float32)[:, 1].astype(np.float64)
    f[:, 96], f[:, 97], f[:, 98], f[:, 99] = np.cos(phi), np.sin(phi), np.sin(th), np.cos(th)
    return bf16(f) if rounding else f


def forward(w, pts, sun, centre, inv_half, rounding=True):
    P = unpack(w)
    R = bf16 if rounding else (lambda x: np.asarray(x, np.float64))
    f = features(pts, sun, centre, inv_half, rounding)
    W1, W2, W3, w4 = R(P["W1"]), R(P["W2"]), R(P["W3"]), R(P["w4"])
    a1 = f @ W1.T + P["b1"]
    h1 = R(np.maximum(a1, 0.0))
    a2 = h1 @ W2.T + P["b2"]
    h2 = R(np.maximum(a2, 0.0))
    a3 = h2 @ W3.T + P["b3"]
    h3 = R(np.maximum(a3, 0.0))
    logit = h3 @ w4 + P["b4"][0]
    cache = dict(f=f, h1=h1, h2=h2, h3=h3, W1=W1, W2=W2, W3=W3, w4=w4, rounding=rounding)
    return logit, cache


def backward(cache, dlogit):
    """Gradient of sum_i dlogit_i * logit_i with respect to the FP32 master parameters
    (straight through the BF16 weight copies)."""
    R = bf16 if cache["rounding"] else (lambda x: np.asarray(x, np.float64))
    dlogit = np.asarray(dlogit, np.float64)
    g = {}
    g["w4"] = dlogit @ cache["h3"]
    g["b4"] = np.array([dlogit.sum()])
    dh3 = np.outer(dlogit, cache["w4"])
    da3 = R(dh3 * (cache["h3"] > 0))
    g["W3"] = da3.T @ cache["h2"]
    g["b3"] = da3.sum(0)
    dh2 = da3 @ cache["W3"]
    da2 = R(dh2 * (cache["h2"] > 0))
    g["W2"] = da2.T @ cache["h1"]
    g["b2"] = da2.sum(0)
    dh1 = da2 @ cache["W2"]
    da1 = R(dh1 * (cache["h1"] > 0))
    g["W1"] = da1.T @ cache["f"]
    g["b1"] = da1.sum(0)
    return pack(g)


def bce_grad(w, pts, sun, labels, centre, inv_half, rounding=True):
    """Mean binary cross-entropy with logits and its gradient."""
    logit, cache = forward(w, pts, sun, centre, inv_half, rounding)
    y = np.asarray(labels, np.float64)
    M = logit.shape[0]
    loss = np.mean(np.maximum(logit, 0) - logit * y + np.log1p(np.exp(-np.abs(logit))))
    dlogit = (1.0 / (1.0 + np.exp(-logit)) - y) / M
    return loss, backward(cache, dlogit), logit


def adam(w, m, v, g, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on FP32 master weights; t counts from 1."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed=0):
    """He-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    d = {}
    for k, s in SIZES.items():
        if k.startswith("b"):
            d[k] = np.zeros(s)
        else:
            fan_in = s[-1] if len(s) == 2 else WIDTH
            lim = np.sqrt(6.0 / fan_in)
            d[k] = rng.uniform(-lim, lim, size=s)
    return pack(d).astype(np.float32)
