"""Synthetic camera-robustness experiment (Sec. 4 "Camera Optimization Robustness"): every
view's 2x4 affine camera is perturbed by a random matrix of Frobenius norm `magnitude` in
normalised coordinates (world scaled to a unit half extent, image mapped to [-1, 1]), the
targets are rendered with the true cameras, and the camera deltas are recovered by Adam on
the L1 image loss with the surfels held fixed.  The residual camera error after the
descent, relative to the injected one, shows how much of the error the camera
optimisation removes.  Every step runs in the library (forward, L1 loss, backward, Adam).
"""
from __future__ import annotations

import numpy as np
import torch

from . import train as tr
from .raster import Context, Plan, default_settings
from .scene_io import scene_to_device


def normalised_scene(scene):
    """The same scene in normalised world coordinates (metres / half extent): surfel
    centres, scales, altitudes and the camera's metric columns rescaled so that every
    pixel sees exactly what it saw before."""
    half = float(scene["spec"].extent) / 2.0
    s = scene["surfels"]
    surf = dict(s, mean=(s["mean"] / half).astype(np.float32), scale=(s["scale"] / half).astype(np.float32))
    F = scene["Fxy"].astype(np.float64).copy()
    F[:, :, :3] *= half
    dF = None if scene.get("dF") is None else np.zeros_like(scene["dF"])
    return dict(scene, surfels=surf, Fxy=F.astype(np.float32), dF=dF,
                b_z=float(np.float32(scene["b_z"] / half)))


def camera_robustness(scene, magnitudes=(1e-3, 4e-3, 1e-2, 4e-2, 1e-1), steps=300, lr0=0.5,
                      decay=0.985, seed=0, ctx=None, tile=8, log=None):
    """Returns one dict per magnitude: injected and recovered camera error (Frobenius, in
    normalised units, mean over views), their ratio, and the L1 loss before / after."""
    ctx = ctx or Context(0)
    sc = normalised_scene(scene)
    surf, views = scene_to_device(sc, with_sun=False)
    W, H = np.asarray(sc["width"]), np.asarray(sc["height"])
    V = len(W)
    plan = Plan(ctx, surf.mean.shape[0], W, H, default_settings(tile_size=tile, batch_depth=64))
    plan.ensure_capacity(surf, views)
    target = plan.forward(surf, views)["image"].clone()
    # pixels per normalised image unit, per row of F (x rows by W/2, y rows by H/2)
    ndc = np.stack([W / 2.0, H / 2.0], 1)[:, :, None]
    F_true = views.Fxy.clone()
    rng = np.random.default_rng(seed)
    out = []
    weights = tr.LossWeights(l1=1.0, normal=0.0, distortion=0.0)
    for mu in magnitudes:
        N = rng.standard_normal((V, 2, 4))
        E = mu * N / np.linalg.norm(N.reshape(V, -1), axis=1)[:, None, None]      # normalised units
        views.Fxy = (F_true + torch.as_tensor((E * ndc).astype(np.float32), device=F_true.device)).contiguous()
        views.dF = torch.zeros(V, 2, 4, dtype=torch.float32, device=F_true.device)
        plan.ensure_capacity(surf, views)
        cfg = tr.adam_config(lr_mean=0.0, lr_scale=0.0, lr_opacity=0.0, lr_quat=0.0, lr_albedo=0.0,
                             lr_dF=lr0, lr_colour=0.0, eps=1e-8, camera_start=1)
        trainer = tr.Trainer(plan, surf, views, target, depth_scale=1.0, cfg=cfg, weights=weights)
        l1_first = None
        for k in range(steps):
            cfg.lr_dF = lr0 * decay ** k
            l1 = float(trainer.step()[0].sum())
            l1_first = l1 if l1_first is None else l1_first
        with torch.no_grad():
            l1_last = float(tr.image_loss_l1(plan, plan.forward(surf, views)["image"], target, 1.0,
                                             torch.empty_like(target)).sum())
        resid = ((views.Fxy + views.dF - F_true).cpu().numpy().astype(np.float64)) / ndc
        err_after = float(np.mean(np.linalg.norm(resid.reshape(V, -1), axis=1)))
        row = dict(magnitude=mu, error_before=float(mu), error_after=err_after,
                   ratio=err_after / mu, l1_before=l1_first, l1_after=l1_last, steps=steps)
        if log:
            log(f"[camera] magnitude {mu:g}: residual {err_after:.3g} ({err_after / mu:.3f} of the "
                f"injected error), L1 {l1_first:.4f} -> {l1_last:.4f}")
        out.append(row)
    views.Fxy = F_true
    return out
