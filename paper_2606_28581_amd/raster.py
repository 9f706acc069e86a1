"""PyTorch-facing wrapper of the C ABI: device memory, streams and autograd plumbing.

Tensors are passed as raw device pointers on torch's current HIP stream; every
computation happens in libsatsplat.so.  Paper: SatSplat (arXiv 2606.28581), Sec. 3.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Dict, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import RasterSettings, StepIO, Surfels, Views, call


def geom_io(depth_scale: float, dist=None, aux=None, d_dist=None):
    g = _lib.GeomIO()
    g.struct_size = C.sizeof(_lib.GeomIO)
    g.depth_scale = float(depth_scale)
    g.dist, g.aux, g.d_dist = _ptr(dist), _ptr(aux), _ptr(d_dist)
    return g


def default_settings(**overrides) -> RasterSettings:
    s = RasterSettings()
    _lib.load().ss_default_settings(C.byref(s))
    for k, v in overrides.items():
        setattr(s, k, v)
    return s


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("satsplat: tensors must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("satsplat: tensors must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """One HIP device (must be gfx950)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        call("ss_context_create", device, C.byref(h))
        self.handle = h
        self.device = device

    def __del__(self):
        if getattr(self, "handle", None) and _lib._lib is not None:
            _lib._lib.ss_context_destroy(self.handle)
            self.handle = None


@dataclass
class SurfelTensors:
    mean: torch.Tensor
    t_u: torch.Tensor
    t_v: torch.Tensor
    scale: torch.Tensor
    opacity: torch.Tensor
    albedo: torch.Tensor

    def c(self) -> Surfels:
        return Surfels(self.mean.shape[0], _ptr(self.mean), _ptr(self.t_u), _ptr(self.t_v),
                       _ptr(self.scale), _ptr(self.opacity), _ptr(self.albedo))


@dataclass
class ViewTensors:
    width: np.ndarray
    height: np.ndarray
    Fxy: torch.Tensor
    b_z: float
    dF: Optional[torch.Tensor] = None
    colC: Optional[torch.Tensor] = None
    colc: Optional[torch.Tensor] = None
    ambient: Optional[torch.Tensor] = None
    sun: Optional[torch.Tensor] = None
    _w: object = field(default=None, repr=False)
    _h: object = field(default=None, repr=False)

    def c(self) -> Views:
        n = int(len(self.width))
        self._w = (C.c_int32 * n)(*[int(x) for x in self.width])
        self._h = (C.c_int32 * n)(*[int(x) for x in self.height])
        return Views(n, self._w, self._h, _ptr(self.Fxy), _ptr(self.dF), _ptr(self.colC),
                     _ptr(self.colc), _ptr(self.ambient), _ptr(self.sun), float(self.b_z))

    @property
    def pixels(self) -> int:
        return int(np.sum(np.asarray(self.width, np.int64) * np.asarray(self.height, np.int64)))


class Plan:
    """Plan + workspace for fixed surfel count and view sizes.  The workspace is a torch
    uint8 tensor; capacities grow on demand (x1.25 of the measured pair counts)."""

    def __init__(self, ctx: Context, n: int, width: Sequence[int], height: Sequence[int],
                 settings: Optional[RasterSettings] = None):
        self.ctx = ctx
        self.settings = settings or default_settings()
        self.n = int(n)
        self.width = np.asarray(width, np.int32)
        self.height = np.asarray(height, np.int32)
        nv = len(self.width)
        w = (C.c_int32 * nv)(*[int(x) for x in self.width])
        h = (C.c_int32 * nv)(*[int(x) for x in self.height])
        ph = C.c_void_p()
        call("ss_plan_create", ctx.handle, self.n, nv, w, h, C.byref(self.settings), C.byref(ph))
        self.handle = ph
        self.cap_main = -1
        self.cap_sun = -1
        self.workspace = None
        self.regrows = 0
        self.bind(0, 0)

    def __del__(self):
        if getattr(self, "handle", None) and _lib._lib is not None:
            _lib._lib.ss_plan_destroy(self.handle)
            self.handle = None

    def set_settings(self, settings: RasterSettings):
        call("ss_plan_set_settings", self.handle, C.byref(settings))
        self.settings = settings

    def workspace_size(self, main_pairs: int, sun_pairs: int) -> int:
        b = C.c_size_t()
        call("ss_plan_workspace_size", self.handle, int(main_pairs), int(sun_pairs), C.byref(b))
        return b.value

    def bind(self, main_pairs: int, sun_pairs: int):
        if main_pairs == self.cap_main and sun_pairs == self.cap_sun:
            return
        nbytes = self.workspace_size(main_pairs, sun_pairs)
        self.workspace = None
        self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8,
                                     device=f"cuda:{self.ctx.device}")
        call("ss_plan_bind_workspace", self.handle, C.c_void_p(self.workspace.data_ptr()),
             self.workspace.numel(), int(main_pairs), int(sun_pairs))
        self.cap_main, self.cap_sun = int(main_pairs), int(sun_pairs)

    def count_pairs(self, s: SurfelTensors, v: ViewTensors):
        m = C.c_int64()
        sp = C.c_int64()
        sc, vc = s.c(), v.c()
        call("ss_count_pairs", self.handle, C.byref(sc), C.byref(vc), C.byref(m), C.byref(sp),
             _stream())
        return m.value, sp.value

    def ensure_capacity(self, s: SurfelTensors, v: ViewTensors, slack: float = 1.25):
        m, sp = self.count_pairs(s, v)
        need_m = max(self.cap_main, int(np.ceil(m * slack)) + 1024) if m > self.cap_main else self.cap_main
        need_s = max(self.cap_sun, int(np.ceil(sp * slack)) + 1024) if sp > self.cap_sun else self.cap_sun
        if need_m != self.cap_main or need_s != self.cap_sun:
            self.bind(need_m, need_s)
        return m, sp

    def check(self):
        o = C.c_int32()
        m = C.c_int64()
        sp = C.c_int64()
        call("ss_plan_check", self.handle, C.byref(o), C.byref(m), C.byref(sp), _stream())
        return bool(o.value), m.value, sp.value

    # ------------------------------------------------------------------ raw calls
    def forward(self, s: SurfelTensors, v: ViewTensors, vis: Optional[torch.Tensor] = None,
                out: Optional[Dict[str, torch.Tensor]] = None, check: bool = True,
                depth_scale: Optional[float] = None):
        """ss_forward; with depth_scale, ss_forward_geom: out also holds the per-pixel
        depth distortion 'dist' and the state 'dist_aux' its backward needs."""
        P = v.pixels
        dev = s.mean.device
        if out is None:
            f = lambda *shape: torch.empty(*shape, dtype=torch.float32, device=dev)
            out = dict(image=f(3 * P), albedo=f(3 * P), vis=f(P), depth=f(P), normal=f(3 * P),
                       T=f(P), last=torch.empty(P, dtype=torch.int32, device=dev))
        if depth_scale is not None and "dist" not in out:
            out["dist"] = torch.empty(P, dtype=torch.float32, device=dev)
            out["dist_aux"] = torch.empty(3 * P, dtype=torch.float32, device=dev)
        for attempt in range(3):
            sc, vc = s.c(), v.c()
            args = (self.handle, C.byref(sc), C.byref(vc), _ptr(vis),
                    _ptr(out["image"]), _ptr(out["albedo"]), _ptr(out["vis"]), _ptr(out["depth"]),
                    _ptr(out["normal"]), _ptr(out["T"]), _ptr(out["last"]))
            if depth_scale is None:
                call("ss_forward", *args, _stream())
            else:
                gio = geom_io(depth_scale, out["dist"], out["dist_aux"])
                call("ss_forward_geom", *args, C.byref(gio), _stream())
            if not check:
                break
            over, m, _ = self.check()
            if not over:
                break
            self.regrows += 1
            self.bind(max(int(m * 1.25) + 1024, self.cap_main), max(self.cap_sun, 0))
        return out

    def backward(self, s: SurfelTensors, v: ViewTensors, fwd: Dict[str, torch.Tensor],
                 d_image=None, d_depth=None, d_normal=None, vis=None, grads=None,
                 depth_scale: Optional[float] = None, d_dist=None):
        """ss_backward; with depth_scale, ss_backward_geom (adds the adjoint of the depth
        distortion for the upstream gradient d_dist, from the forward's 'dist_aux')."""
        n, nv = s.mean.shape[0], len(v.width)
        dev = s.mean.device
        if grads is None:
            z = lambda *shape: torch.empty(*shape, dtype=torch.float32, device=dev)
            grads = dict(mean=z(n, 3), t_u=z(n, 3), t_v=z(n, 3), scale=z(n, 2), opacity=z(n),
                         albedo=z(n, 3), dF=z(nv, 2, 4), colC=z(nv, 3, 3), colc=z(nv, 3),
                         ambient=z(nv, 3))
        sc, vc = s.c(), v.c()
        head = (self.handle, C.byref(sc), C.byref(vc), _ptr(vis),
                _ptr(fwd["albedo"]), _ptr(fwd["vis"]), _ptr(fwd["T"]), _ptr(fwd["last"]),
                _ptr(d_image), _ptr(d_depth), _ptr(d_normal))
        tail = [_ptr(grads[k]) for k in ("mean", "t_u", "t_v", "scale", "opacity", "albedo", "dF",
                                         "colC", "colc", "ambient")]
        if depth_scale is None:
            call("ss_backward", *head, *tail, _stream())
        else:
            gio = geom_io(depth_scale, None, fwd["dist_aux"], d_dist)
            call("ss_backward_geom", *head, C.byref(gio), *tail, _stream())
        return grads

    def normal_loss(self, v: ViewTensors, fwd: Dict[str, torch.Tensor], weight: float = 1.0,
                    tau: float = 0.5, d_depth=None, d_normal=None, d_dF=None,
                    normal_d: bool = False):
        """ss_normal_loss on the forward's depth, T and normal maps.  Returns (loss per
        view, d_depth, d_normal, d_dF, depth normals or None); the gradients are added to
        the given buffers (zeros when None)."""
        P, nv = v.pixels, len(v.width)
        dev = fwd["depth"].device
        z = lambda *shape: torch.zeros(*shape, dtype=torch.float32, device=dev)
        d_depth = z(P) if d_depth is None else d_depth
        d_normal = z(3 * P) if d_normal is None else d_normal
        d_dF = z(nv, 2, 4) if d_dF is None else d_dF
        loss = torch.empty(nv, dtype=torch.float32, device=dev)
        Nd = torch.empty(3 * P, dtype=torch.float32, device=dev) if normal_d else None
        vc = v.c()
        call("ss_normal_loss", self.handle, C.byref(vc), _ptr(fwd["depth"]), _ptr(fwd["T"]),
             _ptr(fwd["normal"]), float(weight), float(tau), _ptr(loss), _ptr(Nd),
             _ptr(d_depth), _ptr(d_normal), _ptr(d_dF), _stream())
        return loss, d_depth, d_normal, d_dF, Nd

    def shadow(self, s: SurfelTensors, v: ViewTensors, vis_out=None, sun_depth=None,
               check: bool = True):
        n, nv = s.mean.shape[0], len(v.width)
        if vis_out is None:
            vis_out = torch.empty(nv, n, dtype=torch.float32, device=s.mean.device)
        for attempt in range(3):
            sc, vc = s.c(), v.c()
            call("ss_shadow_plain", self.handle, C.byref(sc), C.byref(vc), _ptr(sun_depth),
                 _ptr(vis_out), _stream())
            if not check:
                break
            over, _, sp = self.check()
            if not over:
                break
            self.regrows += 1
            self.bind(self.cap_main, max(int(sp * 1.25) + 1024, self.cap_sun))
        return vis_out

    def debug_binning(self, which: int = 0, records: bool = False):
        nt = C.c_int64()
        npairs = C.c_int64()
        call("ss_debug_binning", self.handle, which, None, None, None, None, None,
             C.byref(nt), C.byref(npairs), _stream())
        dev = f"cuda:{self.ctx.device}"
        nv = len(self.width)
        order = torch.empty(self.n, dtype=torch.int32, device=dev)
        tiles = torch.empty(nv, self.n, 4, dtype=torch.int32, device=dev)
        ranges = torch.empty(nt.value, 2, dtype=torch.int32, device=dev)
        lists = torch.empty(max(npairs.value, 1), dtype=torch.int32, device=dev)
        rec = torch.empty(nv, self.n, 24, dtype=torch.float32, device=dev) if records else None
        call("ss_debug_binning", self.handle, which, _ptr(order), _ptr(tiles), _ptr(ranges),
             _ptr(lists), _ptr(rec), C.byref(nt), C.byref(npairs), _stream())
        out = dict(order=order.cpu().numpy().view(np.uint32), tiles=tiles.cpu().numpy(),
                   ranges=ranges.cpu().numpy().view(np.uint32),
                   lists=lists[:npairs.value].cpu().numpy().view(np.uint32))
        if records:
            out["records"] = rec.cpu().numpy()
        return out

    def set_timing(self, on: bool = True):
        call("ss_plan_set_timing", self.handle, 1 if on else 0)

    def read_timing(self):
        """{stage: (total ms, launches)} since the last read (blocks)."""
        ms = (C.c_double * _lib.SS_NUM_STAGES)()
        cnt = (C.c_int64 * _lib.SS_NUM_STAGES)()
        call("ss_plan_read_timing", self.handle, C.cast(ms, C.c_void_p), C.cast(cnt, C.c_void_p))
        lib = _lib.load()
        return {lib.ss_stage_name(k).decode(): (ms[k], cnt[k]) for k in range(_lib.SS_NUM_STAGES)}

    def stats(self):
        out = (C.c_int64 * 7)()
        call("ss_plan_stats", self.handle, C.cast(out, C.c_void_p), _stream())
        keys = ("pairs", "contrib", "evaluated", "sun_pairs", "sun_contrib", "sun_evaluated",
                "fallback")
        return dict(zip(keys, list(out)))

    def debug_sun_cameras(self):
        nv = len(self.width)
        buf = (C.c_double * (9 * nv))()
        call("ss_debug_sun_cameras", self.handle, C.cast(buf, C.c_void_p), _stream())
        return np.frombuffer(buf, dtype=np.float64).reshape(nv, 9).copy()


class StepBuffers:
    """Every device buffer one whole step (shadow pass, forward, backward) touches."""

    def __init__(self, n: int, width, height, device="cuda:0", with_sun=True, sun_map=1024,
                 upstream=None):
        P = int(np.sum(np.asarray(width, np.int64) * np.asarray(height, np.int64)))
        nv = len(width)
        f = lambda *shape: torch.empty(*shape, dtype=torch.float32, device=device)
        self.vis = f(nv, n) if with_sun else None
        self.sun_depth = None
        self.out = dict(image=f(3 * P), albedo=f(3 * P), vis=f(P), depth=f(P), normal=f(3 * P),
                        T=f(P), last=torch.empty(P, dtype=torch.int32, device=device))
        self.grads = dict(mean=f(n, 3), t_u=f(n, 3), t_v=f(n, 3), scale=f(n, 2), opacity=f(n),
                          albedo=f(n, 3), dF=f(nv, 2, 4), colC=f(nv, 3, 3), colc=f(nv, 3),
                          ambient=f(nv, 3))
        self.upstream = upstream or (None, None, None)

    def c(self) -> StepIO:
        o, g = self.out, self.grads
        dI, dD, dN = self.upstream
        io = StepIO()
        io.struct_size = C.sizeof(StepIO)
        vals = dict(vis=self.vis, sun_depth=self.sun_depth, image=o["image"],
                    albedo_out=o["albedo"], vis_out=o["vis"], depth=o["depth"],
                    normal=o["normal"], T_final=o["T"], last=o["last"], d_image=dI, d_depth=dD,
                    d_normal=dN, d_mean=g["mean"], d_t_u=g["t_u"], d_t_v=g["t_v"],
                    d_scale=g["scale"], d_opacity=g["opacity"], d_albedo=g["albedo"],
                    d_dF=g["dF"], d_colC=g["colC"], d_colc=g["colc"], d_ambient=g["ambient"])
        for k, t in vals.items():
            setattr(io, k, None if t is None else _ptr(t).value)
        return io


class Graph:
    """A captured whole step (HIP graph) replayed on torch's current stream."""

    def __init__(self, plan: "Plan", s: SurfelTensors, v: ViewTensors, bufs: StepBuffers):
        h = C.c_void_p()
        self.plan = plan
        self._keep = (s, v, bufs)
        sc, vc, io = s.c(), v.c(), bufs.c()
        call("ss_graph_build", plan.handle, C.byref(sc), C.byref(vc), C.byref(io), C.byref(h))
        self.handle = h

    def launch(self, check: bool = False):
        """Replay the step.  With check=True, block and raise if the replay needed more
        (tile, surfel) pairs than the plan's capacity (its outputs are then incomplete)."""
        call("ss_graph_launch", self.handle, _stream())
        if check and self.plan.check()[0]:
            raise RuntimeError("satsplat: pair capacity overflow in a graph replay; rebind a "
                               "larger workspace and rebuild the graph")

    def __del__(self):
        if getattr(self, "handle", None) and _lib._lib is not None:
            _lib._lib.ss_graph_destroy(self.handle)
            self.handle = None


def step(plan: "Plan", s: SurfelTensors, v: ViewTensors, bufs: StepBuffers):
    sc, vc, io = s.c(), v.c(), bufs.c()
    call("ss_step", plan.handle, C.byref(sc), C.byref(vc), C.byref(io), _stream())


def autotune(plan: "Plan", s: SurfelTensors, v: ViewTensors, bufs: StepBuffers, reps: int = 3):
    """Bind capacities for the largest pair count (tile 8), time all 12 candidates, leave
    the plan on the fastest.  Returns (settings, ms, table)."""
    base = plan.settings
    probe = default_settings(**{k: getattr(base, k) for k, _ in RasterSettings._fields_
                                if k != "struct_size"})
    probe.tile_size = 8
    plan.set_settings(probe)
    plan.ensure_capacity(s, v)
    best = RasterSettings()
    ms = C.c_double()
    table = (C.c_double * 36)()
    sc, vc, io = s.c(), v.c(), bufs.c()
    call("ss_autotune", plan.handle, C.byref(sc), C.byref(vc), C.byref(io), int(reps),
         C.byref(best), C.byref(ms), C.cast(table, C.c_void_p), _stream())
    plan.settings = best
    return best, ms.value, np.frombuffer(table, dtype=np.float64).reshape(12, 3).copy()


class RasterizeAffine2DGS(torch.autograd.Function):
    """Differentiable render of all views: (surfel params, dF, colour terms) ->
    (image, depth, normal).  The backward is the library's hand-written adjoint."""

    @staticmethod
    def forward(ctx, plan: Plan, views: ViewTensors, vis, mean, t_u, t_v, scale, opacity,
                albedo, dF, colC, colc, ambient):
        s = SurfelTensors(mean, t_u, t_v, scale, opacity, albedo)
        v = ViewTensors(views.width, views.height, views.Fxy, views.b_z, dF, colC, colc, ambient,
                        views.sun)
        out = plan.forward(s, v, vis)
        ctx.plan, ctx.views = plan, v
        ctx.has = (colC is not None, colc is not None, ambient is not None)
        ctx.save_for_backward(mean, t_u, t_v, scale, opacity, albedo, vis, out["albedo"],
                              out["vis"], out["T"], out["last"])
        ctx.mark_non_differentiable(out["albedo"], out["vis"], out["T"], out["last"])
        return out["image"], out["depth"], out["normal"], out["albedo"], out["vis"], out["T"], \
            out["last"]

    @staticmethod
    def backward(ctx, d_image, d_depth, d_normal, *_):
        mean, t_u, t_v, scale, opacity, albedo, vis, A, V, T, last = ctx.saved_tensors
        s = SurfelTensors(mean, t_u, t_v, scale, opacity, albedo)
        c = lambda t: None if t is None else t.contiguous()
        fwd = dict(albedo=A, vis=V, T=T, last=last)
        g = ctx.plan.backward(s, ctx.views, fwd, c(d_image), c(d_depth), c(d_normal), vis=vis)
        hC, hc, ha = ctx.has
        return (None, None, None, g["mean"], g["t_u"], g["t_v"], g["scale"], g["opacity"],
                g["albedo"], g["dF"] if ctx.views.dF is not None else None,
                g["colC"] if hC else None, g["colc"] if hc else None,
                g["ambient"] if ha else None)


def rasterize(plan: Plan, views: ViewTensors, surfels: SurfelTensors, vis=None):
    """Autograd entry point.  Returns dict(image [3P], depth [P], normal [3P], albedo,
    vis, T, last) with per-view planar layouts concatenated over views."""
    outs = RasterizeAffine2DGS.apply(plan, views, vis, surfels.mean, surfels.t_u, surfels.t_v,
                                     surfels.scale, surfels.opacity, surfels.albedo, views.dF,
                                     views.colC, views.colc, views.ambient)
    keys = ("image", "depth", "normal", "albedo", "vis", "T", "last")
    return dict(zip(keys, outs))
