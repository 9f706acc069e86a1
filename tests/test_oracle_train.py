"""Pins of the training-step oracle (oracle/train.py): surfel activations and their
adjoint, Adam, and the L1 image loss (Supp. B "Experimental Settings")."""
import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import train as ot


def test_quaternion_frame_special_cases_and_library_rotation():
    R = ot.quat_frame(np.array([[1.0, 0, 0, 0], [np.cos(np.pi / 4), 0, 0, np.sin(np.pi / 4)],
                                [0.0, 0, 0, 3.0]]))
    np.testing.assert_allclose(R[0], np.eye(3), atol=1e-15)
    # 90 degrees about z: x -> y, y -> -x
    np.testing.assert_allclose(R[1][:, 0], [0, 1, 0], atol=1e-15)
    np.testing.assert_allclose(R[1][:, 1], [-1, 0, 0], atol=1e-15)
    # 180 degrees about z, any norm
    np.testing.assert_allclose(R[2][:, 0], [-1, 0, 0], atol=1e-15)
    q = np.random.default_rng(0).standard_normal((50, 4)) * 2.0
    R = ot.quat_frame(q)
    ref = Rotation.from_quat(np.concatenate([q[:, 1:], q[:, :1]], 1)).as_matrix()   # scalar last
    np.testing.assert_allclose(R, ref, atol=1e-13)
    np.testing.assert_allclose(np.einsum("nij,nik->njk", R, R), np.broadcast_to(np.eye(3), R.shape),
                               atol=1e-13)


def test_activation_adjoint_matches_central_differences():
    rng = np.random.default_rng(1)
    n = 7
    raw = rng.standard_normal((n, ot.RAW))
    raw[:, 3:5] *= 0.5
    g = {k: rng.standard_normal(s) for k, s in (("mean", (n, 3)), ("t_u", (n, 3)), ("t_v", (n, 3)),
                                                 ("scale", (n, 2)), ("opacity", (n,)), ("albedo", (n, 3)))}

    def f(r):
        a = ot.activate(r)
        return sum((a[k] * g[k]).sum() for k in g)

    gr = ot.activation_adjoint(raw, g)
    h = 1e-6
    for i in range(n):
        for j in range(ot.RAW):
            rp, rm = raw.copy(), raw.copy()
            rp[i, j] += h
            rm[i, j] -= h
            fd = (f(rp) - f(rm)) / (2 * h)
            assert abs(fd - gr[i, j]) < 1e-7 * max(1.0, abs(fd)), (i, j, fd, gr[i, j])


def test_adam_matches_closed_form_first_step_and_torch():
    cfg = ot.AdamConfig(eps=1e-8)
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(20)
    g = rng.standard_normal(20)
    t1, m, v = ot.adam(theta, np.zeros(20), np.zeros(20), g, 0.01, 1, cfg)
    np.testing.assert_allclose(t1, theta - 0.01 * np.sign(g), atol=1e-9)
    # five steps against torch.optim.Adam on the same gradient sequence
    p = torch.tensor(theta, requires_grad=True)
    opt = torch.optim.Adam([p], lr=0.01, betas=(cfg.beta1, cfg.beta2), eps=cfg.eps)
    th, m, v = theta.copy(), np.zeros(20), np.zeros(20)
    for t in range(1, 6):
        gt = rng.standard_normal(20)
        p.grad = torch.tensor(gt)
        opt.step()
        th, m, v = ot.adam(th, m, v, gt, 0.01, t, cfg)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_l1_loss_closed_form():
    img = np.array([0.5, 0.2, 0.9, 0.1, 0.0, 1.0, 0.3, 0.3, 0.3], np.float64)   # view 0: 1x1, view 1: 2x1
    tgt = np.array([0.4, 0.4, 0.9, 0.2, 0.1, 0.5, 0.3, 0.6, 0.0], np.float64)
    loss, grad = ot.l1_loss(img, tgt, [1, 2], [1, 1], weight=0.8)
    np.testing.assert_allclose(loss, [0.8 * (0.1 + 0.2) / 3, 0.8 * (0.1 + 0.1 + 0.5 + 0.0 + 0.3 + 0.3) / 6])
    np.testing.assert_allclose(grad, 0.8 * np.array([1 / 3, -1 / 3, 0, -1 / 6, -1 / 6, 1 / 6, 0, -1 / 6, 1 / 6]))
