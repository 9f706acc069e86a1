"""Training step over the C ABI (argument marshalling and call order only; every step
runs in libsatsplat.so): raw surfel parameters and Adam moments on the device, the
visibility from the plain shadow pass or the learned surrogate, the forward with the
depth-distortion channel, the L1 image loss, the depth-normal consistency loss, the
backward, and Adam over the surfels, camera deltas and colour terms (Supp. B:
learning rates, loss weights and the camera start step are the paper's defaults).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import call
from .raster import Plan, SurfelTensors, ViewTensors, _ptr, _stream


@dataclass
class LossWeights:
    l1: float = 0.8
    normal: float = 0.05
    distortion: float = 0.05
    tau: float = 0.5          # coverage a pixel needs to enter the normal loss


def adam_config(lr_mean=0.075, lr_scale=0.001, lr_opacity=0.001, lr_quat=0.001,
                lr_albedo=0.0025, lr_dF=0.0001, lr_colour=0.001, beta1=0.9, beta2=0.999,
                eps=1e-15, camera_start=3000) -> _lib.AdamConfig:
    c = _lib.AdamConfig()
    c.struct_size = C.sizeof(_lib.AdamConfig)
    c.lr_mean, c.lr_scale, c.lr_opacity, c.lr_quat = lr_mean, lr_scale, lr_opacity, lr_quat
    c.lr_albedo, c.lr_dF, c.lr_colour = lr_albedo, lr_dF, lr_colour
    c.beta1, c.beta2, c.eps, c.camera_start = beta1, beta2, eps, int(camera_start)
    return c


def surfel_raw(s: SurfelTensors) -> torch.Tensor:
    raw = torch.empty(s.mean.shape[0], _lib.SS_RAW_FLOATS, dtype=torch.float32, device=s.mean.device)
    call("ss_surfel_raw", s.mean.shape[0], _ptr(s.mean), _ptr(s.t_u), _ptr(s.t_v), _ptr(s.scale),
         _ptr(s.opacity), _ptr(s.albedo), _ptr(raw), _stream())
    return raw


def surfel_activate(raw: torch.Tensor, s: SurfelTensors):
    call("ss_surfel_activate", raw.shape[0], _ptr(raw), _ptr(s.mean), _ptr(s.t_u), _ptr(s.t_v),
         _ptr(s.scale), _ptr(s.opacity), _ptr(s.albedo), _stream())


def adam_surfels(raw, m, v, grads, cfg, step, s: SurfelTensors):
    call("ss_adam_surfels", raw.shape[0], _ptr(raw), _ptr(m), _ptr(v),
         *[_ptr(grads[k]) for k in ("mean", "t_u", "t_v", "scale", "opacity", "albedo")],
         C.byref(cfg), int(step), _ptr(s.mean), _ptr(s.t_u), _ptr(s.t_v), _ptr(s.scale),
         _ptr(s.opacity), _ptr(s.albedo), _stream())


def adam_views(v: ViewTensors, state, grads, cfg, step, d_dF_extra=None):
    nv = len(v.width)
    g = lambda k: (_ptr(v.__dict__[k]), _ptr(state["m_" + k]), _ptr(state["v_" + k]), _ptr(grads[k])) \
        if v.__dict__[k] is not None else (None, None, None, None)
    dF, colC, colc = g("dF"), g("colC"), g("colc")
    call("ss_adam_views", nv, *dF, _ptr(d_dF_extra), *colC, *colc, C.byref(cfg), int(step), _stream())


def image_loss_l1(plan: Plan, image, target, weight, d_image, loss=None):
    if loss is None:
        loss = torch.empty(len(plan.width), dtype=torch.float32, device=image.device)
    call("ss_image_loss_l1", plan.handle, _ptr(image), _ptr(target), float(weight), _ptr(loss),
         _ptr(d_image), _stream())
    return loss


class Trainer:
    """Optimises the surfels, camera deltas and colour terms of `views` against `targets`
    (the planar image layout of ss_forward).  `vis` is the visibility input of the
    forward ([n_views, n] or None); give a callable to recompute it every step (e.g. the
    plain shadow pass or the surrogate on the current surfels)."""

    def __init__(self, plan: Plan, surf: SurfelTensors, views: ViewTensors, targets: torch.Tensor,
                 depth_scale: float, cfg: Optional[_lib.AdamConfig] = None,
                 weights: LossWeights = LossWeights(), vis=None):
        dev = surf.mean.device
        self.plan, self.surf, self.views, self.targets = plan, surf, views, targets
        self.cfg = cfg or adam_config()
        self.w, self.ds, self.vis = weights, float(depth_scale), vis
        self.raw = surfel_raw(surf)
        self.m = torch.zeros_like(self.raw)
        self.v = torch.zeros_like(self.raw)
        nv, P, n = len(views.width), views.pixels, surf.mean.shape[0]
        if views.dF is None:
            views.dF = torch.zeros(nv, 2, 4, dtype=torch.float32, device=dev)
        self.vstate = {}
        for k in ("dF", "colC", "colc"):
            t = views.__dict__[k]
            if t is not None:
                self.vstate["m_" + k] = torch.zeros_like(t)
                self.vstate["v_" + k] = torch.zeros_like(t)
        f = lambda *shape: torch.empty(*shape, dtype=torch.float32, device=dev)
        self.d_image = f(3 * P)
        self.d_depth = torch.zeros(P, dtype=torch.float32, device=dev)
        self.d_normal = torch.zeros(3 * P, dtype=torch.float32, device=dev)
        self.d_dF_normal = torch.zeros(nv, 2, 4, dtype=torch.float32, device=dev)
        # the distortion term is weight * mean over each view's pixels: a constant upstream
        self.d_dist = torch.empty(P, dtype=torch.float32, device=dev)
        off = 0
        for w, h in zip(views.width, views.height):
            p = int(w) * int(h)
            self.d_dist[off:off + p].fill_(weights.distortion / p)
            off += p
        self.grads = dict(mean=f(n, 3), t_u=f(n, 3), t_v=f(n, 3), scale=f(n, 2), opacity=f(n),
                          albedo=f(n, 3), dF=f(nv, 2, 4), colC=f(nv, 3, 3), colc=f(nv, 3),
                          ambient=f(nv, 3))
        self.out = None
        self.loss_l1 = torch.empty(nv, dtype=torch.float32, device=dev)
        self.step_count = 0
        # read the plan's overflow flag after every forward (a host synchronisation) and
        # grow the workspace when needed; off for timing loops that check once at the end
        self.check = True

    # ------------------------------------------------------------------ checkpoints
    _VIEW_TERMS = ("dF", "colC", "colc")

    def state_dict(self) -> dict:
        """What a resumed run needs, as host arrays: the raw surfel parameters and their
        Adam moments, the views' learnable terms (camera deltas, colour gain and bias) with
        their moments, and the step count (Adam's bias correction and the camera start
        step count from it)."""
        host = lambda t: t.detach().cpu().numpy().copy()
        d = {"step_count": np.int64(self.step_count), "raw": host(self.raw), "m": host(self.m),
             "v": host(self.v)}
        for k in self._VIEW_TERMS:
            t = self.views.__dict__[k]
            if t is not None:
                d["view_" + k] = host(t)
        for k, t in self.vstate.items():
            d["vstate_" + k] = host(t)
        return d

    def load_state_dict(self, d: dict):
        """Restores a state_dict of a trainer over the same surfel and view counts (and
        the same learnable view terms) in place, then rewrites the activated surfel
        arrays from the raw parameters."""
        def put(dst: torch.Tensor, a, name):
            a = np.asarray(a)
            if tuple(a.shape) != tuple(dst.shape) or a.dtype != np.float32:
                raise ValueError(f"checkpoint entry {name}: {a.dtype}{tuple(a.shape)} does not fit "
                                 f"float32{tuple(dst.shape)}")
            dst.copy_(torch.from_numpy(a))
        put(self.raw, d["raw"], "raw")
        put(self.m, d["m"], "m")
        put(self.v, d["v"], "v")
        for k in self._VIEW_TERMS:
            t = self.views.__dict__[k]
            if (t is None) != ("view_" + k not in d):
                raise ValueError(f"checkpoint and trainer disagree on the view term {k}")
            if t is not None:
                put(t, d["view_" + k], "view_" + k)
        for k, t in self.vstate.items():
            put(t, d["vstate_" + k], "vstate_" + k)
        self.step_count = int(d["step_count"])
        surfel_activate(self.raw, self.surf)
        self.out = None

    def save(self, path):
        """state_dict() into an .npz file (plain arrays, no pickled objects)."""
        np.savez(path, **self.state_dict())

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            self.load_state_dict({k: z[k] for k in z.files})

    def step(self):
        """One training step; returns (per-view L1 loss, per-view normal loss) tensors (the
        L1 buffer is the trainer's own and is overwritten by the next step)."""
        self.step_count += 1
        vis = self.vis() if callable(self.vis) else self.vis
        self.out = self.plan.forward(self.surf, self.views, vis, out=self.out, depth_scale=self.ds,
                                     check=self.check)
        image_loss_l1(self.plan, self.out["image"], self.targets, self.w.l1, self.d_image,
                      self.loss_l1)
        self.d_depth.zero_()
        self.d_normal.zero_()
        self.d_dF_normal.zero_()
        loss_n, *_ = self.plan.normal_loss(self.views, self.out, weight=self.w.normal, tau=self.w.tau,
                                           d_depth=self.d_depth, d_normal=self.d_normal,
                                           d_dF=self.d_dF_normal)
        self.plan.backward(self.surf, self.views, self.out, self.d_image, self.d_depth, self.d_normal,
                           vis=vis, grads=self.grads, depth_scale=self.ds, d_dist=self.d_dist)
        adam_surfels(self.raw, self.m, self.v, self.grads, self.cfg, self.step_count, self.surf)
        adam_views(self.views, self.vstate, self.grads, self.cfg, self.step_count, self.d_dF_normal)
        return self.loss_l1, loss_n
