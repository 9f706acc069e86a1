"""Pins of the MLP-surrogate oracle (oracle/mlp.py): an independent torch-FP64 network,
finite differences, closed-form features, bfloat16 rounding cases, Adam's first step,
and learning a separable toy problem to 100 %."""
import math

import numpy as np
import torch

from oracle import mlp

CENTRE = np.array([1.0, -2.0, 10.0], np.float32)
INV_HALF = np.float32(1.0 / 64.0)


def data(M=64, seed=0):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-60, 60, size=(M, 3)).astype(np.float32) + CENTRE
    sun = np.stack([rng.uniform(0, 2 * np.pi, M), rng.uniform(0.5, 1.2, M)], 1).astype(np.float32)
    return pts, sun


def test_bf16_rounding_cases():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9, 1 + 2 ** -7 + 2 ** -8, -2.5, 3.0e-3])
    r = mlp.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie -> even
    assert r[2] == 1 + 2 ** -7              # above the tie -> up
    assert r[3] == 1 + 2 ** -6              # tie, odd -> up to even
    assert r[4] == -2.5
    assert abs(r[5] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_fourier_features_closed_form():
    pts = (np.array([[0.5, 1 / 3, 0.0]], np.float32) / INV_HALF + CENTRE).astype(np.float32)
    sun = np.array([[math.pi / 6, math.pi / 4]], np.float32)
    f = mlp.features(pts, sun, CENTRE, INV_HALF, rounding=False)[0]
    # x = 0.5: sin(pi/2)=1, cos=0; k=1: sin(pi)=0, cos=-1; k>=2: sin=0, cos=1
    assert abs(f[0] - 1) < 1e-15 and abs(f[1]) < 1e-15
    assert abs(f[2]) < 1e-15 and abs(f[3] + 1) < 1e-15
    for k in range(2, 16):
        assert abs(f[2 * k]) < 1e-12 and abs(f[2 * k + 1] - 1) < 1e-12
    ph = mlp.normalise(pts, CENTRE, INV_HALF)[0, 1].astype(np.float64)
    for k in range(16):
        assert abs(f[32 + 2 * k] - math.sin(math.pi * ph * 2 ** k)) < 1e-9
    assert np.all(f[64:96:2] == 0) and np.all(f[65:96:2] == 1)   # z = 0 exactly
    np.testing.assert_allclose(f[96:100], [math.cos(np.float32(math.pi / 6)), math.sin(np.float32(math.pi / 6)),
                                           math.sin(np.float32(math.pi / 4)), math.cos(np.float32(math.pi / 4))])
    assert np.all(f[100:] == 0)


def torch_net(w, f):
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in mlp.unpack(w).items()}
    x = torch.tensor(f)
    h = torch.relu(torch.nn.functional.linear(x, P["W1"], P["b1"]))
    h = torch.relu(torch.nn.functional.linear(h, P["W2"], P["b2"]))
    h = torch.relu(torch.nn.functional.linear(h, P["W3"], P["b3"]))
    return h @ P["w4"] + P["b4"], P


def test_unrounded_oracle_equals_torch_fp64_network_and_autograd():
    pts, sun = data()
    w = mlp.init_params(1).astype(np.float64) * 0.5
    f = mlp.features(pts, sun, CENTRE, INV_HALF, rounding=False)
    logit, cache = mlp.forward(w, pts, sun, CENTRE, INV_HALF, rounding=False)
    tl, P = torch_net(w, f)
    np.testing.assert_allclose(logit, tl.detach().numpy(), rtol=1e-12, atol=1e-12)
    dl = np.random.default_rng(3).normal(size=logit.shape)
    (tl * torch.tensor(dl)).sum().backward()
    g = mlp.backward(cache, dl)
    gt = mlp.pack({k: v.grad.numpy() for k, v in P.items()})
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-12)


def test_unrounded_gradient_matches_finite_differences():
    pts, sun = data(32, 5)
    w = mlp.init_params(2).astype(np.float64)
    labels = (np.random.default_rng(1).uniform(size=32) > 0.5).astype(np.float64)
    loss, g, _ = mlp.bce_grad(w, pts, sun, labels, CENTRE, INV_HALF, rounding=False)
    rng = np.random.default_rng(7)
    for i in rng.choice(w.size, 40, replace=False):
        h = 1e-6
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        lp = mlp.bce_grad(wp, pts, sun, labels, CENTRE, INV_HALF, rounding=False)[0]
        lm = mlp.bce_grad(wm, pts, sun, labels, CENTRE, INV_HALF, rounding=False)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3), (i, fd, g[i])


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w = np.zeros(4)
    w1, m, v = mlp.adam(w, np.zeros(4), np.zeros(4), g, lr=0.01, t=1)
    np.testing.assert_allclose(w1, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_rounded_network_learns_a_separable_toy_problem():
    rng = np.random.default_rng(4)
    pts = (rng.uniform(-60, 60, size=(256, 3)) + CENTRE).astype(np.float32)
    sun = np.stack([rng.uniform(0, 2 * np.pi, 256), rng.uniform(0.5, 1.2, 256)], 1).astype(np.float32)
    labels = (pts[:, 0] > CENTRE[0]).astype(np.float64)
    w = mlp.init_params(3).astype(np.float64) * 0.3
    m = np.zeros_like(w); v = np.zeros_like(w)
    for t in range(1, 301):
        loss, g, logit = mlp.bce_grad(w, pts, sun, labels, CENTRE, INV_HALF, rounding=True)
        w, m, v = mlp.adam(w, m, v, g, lr=3e-3, t=t)
    logit, _ = mlp.forward(w, pts, sun, CENTRE, INV_HALF, rounding=True)
    assert np.mean((logit > 0) == (labels > 0.5)) == 1.0
