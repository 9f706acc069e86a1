"""Learned sun-visibility surrogate: ctypes plumbing around the MLP entry points of the
C ABI (every step runs in libsatsplat.so)."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import MlpConfig, call
from .raster import Context, Plan, SurfelTensors, ViewTensors, _ptr, _stream

N_PARAMS = _lib.SS_MLP_PARAMS


class Mlp:
    """The surrogate network: normalisation constants + a training workspace."""

    def __init__(self, ctx: Context, centre, inv_half: float, max_points: int | None = 0):
        """max_points=None binds no workspace (only backward_noalloc may then run)."""
        cfg = MlpConfig()
        cfg.struct_size = C.sizeof(MlpConfig)
        for i in range(3):
            cfg.centre[i] = float(centre[i])
        cfg.inv_half = float(inv_half)
        h = C.c_void_p()
        call("ss_mlp_create", ctx.handle, C.byref(cfg), C.byref(h))
        self.handle, self.ctx, self.max_points = h, ctx, 0
        self.workspace = None
        if max_points is not None:
            self.bind(max_points)

    def bind(self, max_points: int):
        b = C.c_size_t()
        call("ss_mlp_workspace_size", self.handle, int(max_points), C.byref(b))
        self.workspace = torch.empty(max(b.value, 256), dtype=torch.uint8,
                                     device=f"cuda:{self.ctx.device}")
        call("ss_mlp_bind_workspace", self.handle, C.c_void_p(self.workspace.data_ptr()),
             self.workspace.numel(), int(max_points))
        self.max_points = int(max_points)

    def __del__(self):
        if getattr(self, "handle", None) and _lib._lib is not None:
            _lib._lib.ss_mlp_destroy(self.handle)
            self.handle = None

    def forward(self, w, pts, sun, all_pairs=False, prob=False, out=None):
        n_pts, n_sun = pts.shape[0], sun.shape[0]
        M = n_pts * n_sun if all_pairs else n_pts
        if out is None:
            out = torch.empty(M, dtype=torch.float32, device=pts.device)
        call("ss_mlp_forward", self.handle, _ptr(w), _ptr(pts), n_pts, _ptr(sun), n_sun,
             1 if all_pairs else 0, 1 if prob else 0, _ptr(out), _stream())
        return out

    def backward(self, w, pts, sun, labels=None, d_logits=None, scale=1.0, d_w=None, loss=None):
        if d_w is None:
            d_w = torch.empty(N_PARAMS, dtype=torch.float32, device=pts.device)
        call("ss_mlp_backward", self.handle, _ptr(w), _ptr(pts), _ptr(sun), pts.shape[0],
             _ptr(labels), _ptr(d_logits), float(scale), _ptr(d_w), _ptr(loss), _stream())
        return d_w

    def backward_noalloc(self, w, pts, sun, labels=None, d_logits=None, scale=1.0, d_w=None,
                         loss=None):
        """ss_mlp_backward_noalloc: the same gradient with the library's fixed scratch array
        instead of this object's workspace (up to SS_NOALLOC_MAX_POINTS points)."""
        if d_w is None:
            d_w = torch.empty(N_PARAMS, dtype=torch.float32, device=pts.device)
        call("ss_mlp_backward_noalloc", self.handle, _ptr(w), _ptr(pts), _ptr(sun), pts.shape[0],
             _ptr(labels), _ptr(d_logits), float(scale), _ptr(d_w), _ptr(loss), _stream())
        return d_w


def save_network(path, centre, inv_half, w, m=None, v=None, step=0):
    """Surrogate checkpoint as an .npz of plain arrays: the normalisation constants the
    network was trained with (Mlp(ctx, centre, inv_half)), its N_PARAMS weights and, to
    resume training, the Adam moments and the step count."""
    host = lambda t: (t.detach().cpu().numpy() if isinstance(t, torch.Tensor) else np.asarray(t)) \
        .astype(np.float32).reshape(-1)
    d = dict(centre=np.asarray(centre, np.float64).reshape(3), inv_half=np.float64(inv_half),
             w=host(w), step=np.int64(step))
    if (m is None) != (v is None):
        raise ValueError("give both Adam moments or neither")
    if m is not None:
        d["m"], d["v"] = host(m), host(v)
    for k in ("w", "m", "v"):
        if k in d and d[k].size != N_PARAMS:
            raise ValueError(f"{k} holds {d[k].size} values, the network has {N_PARAMS}")
    np.savez(path, **d)


def load_network(path, device="cuda") -> dict:
    """A save_network file: centre (3 floats), inv_half, step, and w, m, v as float32
    tensors on `device` (m and v None when the file holds no moments)."""
    with np.load(path, allow_pickle=False) as z:
        if z["w"].size != N_PARAMS:
            raise ValueError(f"checkpoint holds {z['w'].size} weights, the network has {N_PARAMS}")
        t = lambda k: torch.as_tensor(z[k].astype(np.float32), device=device) if k in z.files else None
        return dict(centre=z["centre"].astype(np.float64), inv_half=float(z["inv_half"]),
                    step=int(z["step"]), w=t("w"), m=t("m"), v=t("v"))


def adam(w, m, v, g, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
    call("ss_mlp_adam", _ptr(w), _ptr(m), _ptr(v), _ptr(g), w.numel(), float(lr), float(beta1),
         float(beta2), float(eps), int(step), _stream())


def shadow_surrogate(plan: Plan, mlp: Mlp, w, s: SurfelTensors, v: ViewTensors, band=0.1,
                     vis_out=None, sun_depth=None):
    n, nv = s.mean.shape[0], len(v.width)
    if vis_out is None:
        vis_out = torch.empty(nv, n, dtype=torch.float32, device=s.mean.device)
    sc, vc = s.c(), v.c()
    call("ss_shadow_surrogate", plan.handle, mlp.handle, _ptr(w), C.byref(sc), C.byref(vc),
         float(band), _ptr(vis_out), _ptr(sun_depth), _stream())
    return vis_out
