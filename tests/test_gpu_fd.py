"""Finite differences through the library's forward against its backward, all on the GPU
(end-to-end differentiability of the rasterizer, Sec. 3.5; adjoint of Eq. rasterization
and of the projection, Sec. 3.2-3.3).

The loss is L = <dI, image> + <dD, depth> + <dN, normal> (+ <dd, distortion>) with seeded
upstream weights, summed in FP64 on the host from the FP32 outputs.  The thresholds that
make the forward jump (alpha_min and the T_min stop) are moved out of reach
(alpha_min = T_min = 1e-20; the support boxes grow accordingly), so central differences
see a smooth function; the depth order, a step function of the centres' altitudes, is kept
by moving all altitudes by one common amount.  With the low-pass applied to every surfel
(mode 0) a pixel switches between the surfel's own Gaussian and the low-pass disk where
the two distances are equal, a kink of alpha and a jump of the pair's depth (the centre's
depth on the low-pass branch); mode 0 is therefore checked on the parameter groups that do
not move that boundary, mode 1 (low-pass only for degenerate surfels) on all.  Per parameter
group the test compares the directional derivative along a seeded random direction: the
change of L between the FP32 parameters theta + eps u and theta - eps u against
<g, (theta + eps u) - (theta - eps u)>, both sides taken on the perturbation actually
stored in FP32."""
import dataclasses

import numpy as np
import pytest
import torch

import synth
import paper_2606_28581_amd as ss
from gpu_common import context, to_np

pytestmark = pytest.mark.gpu

SURF = ("mean", "t_u", "t_v", "scale", "opacity", "albedo")
VIEW = ("dF", "colC", "colc", "ambient")
# relative steps: the outputs are linear in albedo and the colour terms (no truncation
# error, so large steps that lift the change of L far above FP32 rounding)
EPS = {"mean": 2e-3, "t_u": 1e-3, "t_v": 1e-3, "scale": 1e-3, "opacity": 1e-2, "albedo": 0.1,
       "dF": 2e-5, "colC": 0.1, "colc": 0.1, "ambient": 0.1}
# groups that do not move the boundary between the low-pass and the surfel branch
KINK_FREE = ("opacity", "albedo", "colC", "colc", "ambient")


def smooth_plan(sc, ts, mode):
    surf, views = ss.scene_to_device(sc)
    st = ss.default_settings(tile_size=ts, batch_depth=32, lowpass_mode=mode,
                             alpha_min=1e-20, T_min=1e-20)
    plan = ss.Plan(context(), surf.mean.shape[0], views.width, views.height, st)
    plan.ensure_capacity(surf, views)
    return plan, surf, views


def loss(plan, surf, views, vis, up, ds):
    out = plan.forward(surf, views, vis, depth_scale=ds)
    val = sum(float(np.dot(to_np(out[k]).astype(np.float64).ravel(), up[k].astype(np.float64)))
              for k in ("image", "depth", "normal"))
    if ds is not None:
        val += float(np.dot(to_np(out["dist"]).astype(np.float64), up["dist"].astype(np.float64)))
    return val, out


@pytest.mark.parametrize("ts,mode,with_dist,groups", [(8, 1, True, SURF + VIEW),
                                                      (16, 1, False, SURF + VIEW),
                                                      (32, 1, True, SURF + VIEW),
                                                      (8, 0, False, KINK_FREE)])
def test_directional_derivatives_match_central_differences(ts, mode, with_dist, groups):
    sc = synth.make_scene(synth.tiny(n_surfels=80, views=((26, 21), (19, 24)), seed=31))
    ds = float(np.float32(2.0 / sc["spec"].extent)) if with_dist else None
    plan, surf, views = smooth_plan(sc, ts, mode)
    P = views.pixels
    rng = np.random.default_rng(32)
    up = dict(image=rng.standard_normal(3 * P).astype(np.float32),
              depth=(0.05 * rng.standard_normal(P)).astype(np.float32),
              normal=rng.standard_normal(3 * P).astype(np.float32),
              dist=(10.0 * rng.standard_normal(P)).astype(np.float32))
    # visibility in (0, 1] so that the ambient term has a gradient (I uses V + (1 - V) L_a)
    vis = torch.as_tensor(rng.uniform(0.2, 1.0, size=(len(views.width), surf.mean.shape[0]))
                          .astype(np.float32), device="cuda")
    L0, out = loss(plan, surf, views, vis, up, ds)
    cu = lambda a: torch.as_tensor(a, device="cuda")
    g = plan.backward(surf, views, out, cu(up["image"]), cu(up["depth"]), cu(up["normal"]), vis=vis,
                      depth_scale=ds, d_dist=cu(up["dist"]) if ds is not None else None)
    g = {k: to_np(t).astype(np.float64) for k, t in g.items()}
    for name in groups:
        owner = surf if name in SURF else views
        x = to_np(getattr(owner, name))
        u = rng.standard_normal(x.shape)
        if name == "mean":
            # the centres' depth order (by altitude) is a step function of the altitudes,
            # and the flat ground's surfels tie: move every altitude by one common amount,
            # which keeps the order
            u[:, 2] = 0.5
        scale = np.abs(to_np(views.Fxy)).mean() if name == "dF" else np.abs(x).mean()
        h = EPS[name] * max(scale, 1e-3)
        L = []
        for sgn in (1.0, -1.0):
            xs = (x + sgn * h * u).astype(np.float32)
            moved = dataclasses.replace(owner, **{name: cu(xs)})
            L.append((loss(plan, *((moved, views) if name in SURF else (surf, moved)), vis, up, ds)[0], xs))
        (Lp, xp), (Lm, xm) = L
        fd = Lp - Lm
        an = float(np.sum(g[name] * (xp.astype(np.float64) - xm.astype(np.float64))))
        err = abs(fd - an) / max(abs(an), 1e-12)
        print(f"[fd] ts {ts} mode {mode} dist {with_dist} {name}: fd {fd:.6e} analytic {an:.6e} "
              f"rel {err:.2e}", flush=True)
        assert abs(an) > 1e-4 * abs(L0) * EPS[name], (name, an)
        assert err < 1e-2, (name, fd, an)
