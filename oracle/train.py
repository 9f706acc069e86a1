"""FP64 oracle of the training step around the rasterizer (Supp. B "Experimental
Settings"): surfel activations, the L1 image loss, and Adam with per-group learning rates
over the surfels and the per-view camera delta and colour terms, the camera group held
until a start step.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke entry point and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path.

Readings (the paper lists the optimiser, its learning rates and the loss weights, not
the parameterisation):
* raw surfel parameters, 13 floats per surfel: mean (3, metres), log scale (2),
  opacity logit (1), rotation quaternion (w, x, y, z) of any non-zero norm (4), albedo
  (3); activations scale = exp, opacity = sigmoid, frame R = rotation of q / |q| with
  t_u, t_v its first two columns (Sec. 3.1: the normal is R's last column); the albedo is
  optimised directly (no spherical harmonics, Sec. 3.2);
* L1 image loss per view: weight / (3 P) * sum over pixels and channels of |I - I*|,
  gradient weight * sign(I - I*) / (3 P) (sign(0) = 0);
* Adam with bias correction, step t counted from 1: m = b1 m + (1 - b1) g,
  v = b2 v + (1 - b2) g^2, theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
  the camera-delta group is not updated (nor are its moments) before `camera_start`,
  and its bias correction counts its own steps, t - camera_start + 1; the colour gain
  and bias use lr_colour from the first step, the ambient term is not trained.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

RAW = 13   # mean 3, log scale 2, opacity logit 1, quaternion 4, albedo 3


@dataclass
class AdamConfig:
    lr_mean: float = 0.075
    lr_scale: float = 0.001
    lr_opacity: float = 0.001
    lr_quat: float = 0.001
    lr_albedo: float = 0.0025
    lr_dF: float = 0.0001
    lr_colour: float = 0.001
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    camera_start: int = 3000


def group_lr(cfg: AdamConfig):
    """Learning rate of each of the 13 raw surfel floats."""
    return np.array([cfg.lr_mean] * 3 + [cfg.lr_scale] * 2 + [cfg.lr_opacity] +
                    [cfg.lr_quat] * 4 + [cfg.lr_albedo] * 3, np.float64)


def quat_frame(q):
    """Columns of the rotation of q / |q|: R [n, 3, 3] (R[:, :, 0] = t_u, [:, :, 1] = t_v)."""
    q = np.asarray(q, np.float64)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = qn.T
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - w * z); R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y); R[:, 2, 1] = 2 * (y * z + w * x); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def activate(raw):
    raw = np.asarray(raw, np.float64).reshape(-1, RAW)
    R = quat_frame(raw[:, 6:10])
    return dict(mean=raw[:, 0:3].copy(), scale=np.exp(raw[:, 3:5]),
                opacity=1.0 / (1.0 + np.exp(-raw[:, 5])), t_u=R[:, :, 0], t_v=R[:, :, 1],
                albedo=raw[:, 10:13].copy())


def activation_adjoint(raw, g):
    """Gradient w.r.t. the raw parameters [n, 13] from gradients w.r.t. the activated
    ones (dict mean, t_u, t_v, scale, opacity, albedo)."""
    raw = np.asarray(raw, np.float64).reshape(-1, RAW)
    out = np.zeros_like(raw)
    out[:, 0:3] = g["mean"]
    out[:, 3:5] = g["scale"] * np.exp(raw[:, 3:5])
    o = 1.0 / (1.0 + np.exp(-raw[:, 5]))
    out[:, 5] = g["opacity"] * o * (1.0 - o)
    q = raw[:, 6:10]
    nq = np.linalg.norm(q, axis=1, keepdims=True)
    qn = q / nq
    w, x, y, z = qn.T
    gu, gv = np.asarray(g["t_u"], np.float64), np.asarray(g["t_v"], np.float64)
    # d t_u / d(w, x, y, z) and d t_v / d(w, x, y, z), each a 3-vector
    du = [np.stack([0 * w, 2 * z, -2 * y], 1), np.stack([0 * w, 2 * y, 2 * z], 1),
          np.stack([-4 * y, 2 * x, -2 * w], 1), np.stack([-4 * z, 2 * w, 2 * x], 1)]
    dv = [np.stack([-2 * z, 0 * w, 2 * x], 1), np.stack([2 * y, -4 * x, 2 * w], 1),
          np.stack([2 * x, 0 * w, 2 * z], 1), np.stack([-2 * w, -4 * z, 2 * y], 1)]
    gqn = np.stack([(gu * du[k]).sum(1) + (gv * dv[k]).sum(1) for k in range(4)], 1)
    out[:, 6:10] = (gqn - qn * (qn * gqn).sum(1, keepdims=True)) / nq
    out[:, 10:13] = g["albedo"]
    return out


def adam(theta, m, v, g, lr, t, cfg: AdamConfig):
    """One Adam update (arrays broadcast against lr); returns new (theta, m, v)."""
    m = cfg.beta1 * m + (1 - cfg.beta1) * g
    v = cfg.beta2 * v + (1 - cfg.beta2) * g * g
    mh = m / (1 - cfg.beta1 ** t)
    vh = v / (1 - cfg.beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + cfg.eps), m, v


def l1_loss(image, target, widths, heights, weight):
    """Per-view L1 loss and its gradient (planar [3, H, W] per view, concatenated)."""
    image = np.asarray(image, np.float64)
    target = np.asarray(target, np.float64)
    loss = np.zeros(len(widths))
    grad = np.zeros_like(image)
    off = 0
    for k, (w, h) in enumerate(zip(widths, heights)):
        n = 3 * int(w) * int(h)
        d = image[off:off + n] - target[off:off + n]
        loss[k] = weight * np.abs(d).sum() / n
        grad[off:off + n] = weight * np.sign(d) / n
        off += n
    return loss, grad
