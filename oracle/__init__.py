"""FP64 CPU oracle for the SatSplat hot path (arXiv 2606.28581).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke entry point and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP path
(paper_2606_28581_amd); the only common module is the seeded input generator `synth`.

`build()` compiles satsplat_oracle.c with gcc (OpenMP).  The wrappers below widen
nothing themselves: they pass the FP32 input arrays straight to C, which widens them
exactly to FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "satsplat_oracle.c")
LIB = os.path.join(HERE, "libsatsplat_oracle.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-D_DEFAULT_SOURCE", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Settings(C.Structure):
    _fields_ = [("alpha_min", C.c_double), ("alpha_max", C.c_double), ("T_min", C.c_double),
                ("sigma", C.c_double), ("det_rel_eps", C.c_double),
                ("lowpass_mode", C.c_int32), ("esm_c", C.c_double), ("esm_bias", C.c_double),
                ("depth_scale", C.c_double)]


@dataclass
class Settings:
    """Rasterizer constants.  alpha_min = 1/255 and T_min = 1e-4 are the stated
    workload values; the others are readings where the paper is silent."""
    alpha_min: float = np.float32(1.0 / 255.0).item()
    alpha_max: float = np.float32(0.99).item()
    T_min: float = np.float32(1e-4).item()
    sigma: float = np.float32(0.70710678).item()
    det_rel_eps: float = np.float32(1e-6).item()
    lowpass_mode: int = 0
    esm_c: float = 2.0
    esm_bias: float = 0.5
    sun_map_size: int = 1024
    tile_size: int = 16
    depth_scale: float = 1.0     # normalised depth m = z * depth_scale in the distortion

    def c(self):
        return _Settings(self.alpha_min, self.alpha_max, self.T_min, self.sigma,
                         self.det_rel_eps, self.lowpass_mode, self.esm_c, self.esm_bias,
                         self.depth_scale)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = C.CDLL(LIB)
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def _surf_args(s):
    return [_f32(s[k]) for k in ("mean", "t_u", "t_v", "scale", "opacity", "albedo")]


def depth_order(mean, bz):
    mean = _f32(mean)
    n = mean.shape[0]
    out = np.empty(n, np.int64)
    lib().or_depth_order(C.c_int64(n), _p(mean), C.c_float(bz), _p(out))
    return out


def _views(scene):
    W = np.ascontiguousarray(scene["width"], np.int32)
    H = np.ascontiguousarray(scene["height"], np.int32)
    return W, H, _f32(scene["Fxy"]), _f32(scene.get("dF")), _f32(scene.get("colC")), \
        _f32(scene.get("colc")), _f32(scene.get("ambient"))


def forward(scene, settings: Settings = Settings(), vis=None, sel=None, with_dist=False):
    """Render every view (sel None -> full planar CHW layout) or only the global pixel
    indices in `sel` (compact layout).  Returns a dict of float64 arrays; with_dist adds
    the per-pixel depth distortion 'dist'."""
    s = scene["surfels"]
    arrs = _surf_args(s)
    n = arrs[0].shape[0]
    W, H, F, dF, cC, cc, am = _views(scene)
    nv = W.shape[0]
    P = int(np.sum(W.astype(np.int64) * H))
    vis = _f32(vis)
    if sel is not None:
        sel = np.ascontiguousarray(sel, np.int64)
        m = sel.shape[0]
    else:
        m = P
    img = np.zeros(3 * m); A = np.zeros(3 * m); Vo = np.zeros(m); D = np.zeros(m)
    N = np.zeros(3 * m); T = np.zeros(m); cnt = np.zeros(m, np.int64); amb = np.zeros(m, np.uint8)
    sig = np.zeros(m, np.uint64)
    dist = np.zeros(m) if with_dist else None
    st = settings.c()
    L = lib()
    L.or_forward(C.c_int64(n), *[_p(a) for a in arrs], C.c_int32(nv), _p(W), _p(H), _p(F),
                 _p(dF), _p(cC), _p(cc), _p(am), _p(vis), C.c_float(scene["b_z"]),
                 C.byref(st), C.c_int64(m if sel is not None else 0), _p(sel),
                 _p(img), _p(A), _p(Vo), _p(D), _p(N), _p(T), _p(cnt), _p(amb), _p(sig),
                 _p(dist))
    # sig: per-pixel digest of the discrete decisions (contributing surfels, stop, branch,
    # clamp, degenerate flags); equal digests mean the forward is smooth between two inputs
    out = dict(image=img, albedo=A, vis=Vo, depth=D, normal=N, T=T, count=cnt,
               ambiguous=amb.astype(bool), sig=sig)
    if with_dist:
        out["dist"] = dist
    return out


def backward(scene, dI, dD, dN, settings: Settings = Settings(), vis=None, sel=None,
             dDist=None):
    """Adjoint of forward(): upstream gradients of the image [.,3], depth, normal [.,3]
    and (optionally) the per-pixel distortion, in forward()'s layout."""
    s = scene["surfels"]
    arrs = _surf_args(s)
    n = arrs[0].shape[0]
    W, H, F, dF, cC, cc, am = _views(scene)
    nv = W.shape[0]
    vis = _f32(vis)
    m = 0
    if sel is not None:
        sel = np.ascontiguousarray(sel, np.int64)
        m = sel.shape[0]
    g = dict(mean=np.zeros(3 * n), t_u=np.zeros(3 * n), t_v=np.zeros(3 * n),
             scale=np.zeros(2 * n), opacity=np.zeros(n), albedo=np.zeros(3 * n),
             dF=np.zeros(8 * nv), colC=np.zeros(9 * nv), colc=np.zeros(3 * nv),
             ambient=np.zeros(3 * nv))
    st = settings.c()
    lib().or_backward(C.c_int64(n), *[_p(a) for a in arrs], C.c_int32(nv), _p(W), _p(H),
                      _p(F), _p(dF), _p(cC), _p(cc), _p(am), _p(vis), C.c_float(scene["b_z"]),
                      C.byref(st), C.c_int64(m), _p(sel), _p(_f32(dI)), _p(_f32(dD)),
                      _p(_f32(dN)), _p(_f32(dDist)), *[_p(g[k]) for k in ("mean", "t_u", "t_v", "scale",
                                                         "opacity", "albedo", "dF", "colC",
                                                         "colc", "ambient")])
    shapes = dict(mean=(n, 3), t_u=(n, 3), t_v=(n, 3), scale=(n, 2), opacity=(n,),
                  albedo=(n, 3), dF=(nv, 2, 4), colC=(nv, 3, 3), colc=(nv, 3), ambient=(nv, 3))
    return {k: v.reshape(shapes[k]) for k, v in g.items()}


def view_camera(scene, v):
    B = np.zeros(6); b = np.zeros(2)
    lib().or_view_camera(_p(_f32(scene["Fxy"])), _p(_f32(scene.get("dF"))), C.c_int32(v),
                         _p(B), _p(b))
    return B.reshape(2, 3), b


def binning(scene, B, b, W, H, ts, settings: Settings = Settings()):
    """FP64 support boxes -> (c [n,2], h [n,2], pix [n,4], tiles [n,4])."""
    arrs = _surf_args(scene["surfels"])[:5]
    n = arrs[0].shape[0]
    c = np.zeros(2 * n); h = np.zeros(2 * n)
    pix = np.zeros(4 * n, np.int32); tiles = np.zeros(4 * n, np.int32)
    B = np.ascontiguousarray(B, np.float64).ravel(); b = np.ascontiguousarray(b, np.float64)
    st = settings.c()
    lib().or_binning(C.c_int64(n), *[_p(a) for a in arrs], _p(B), _p(b),
                     C.c_float(scene["b_z"]), C.c_int32(W), C.c_int32(H), C.c_int32(ts),
                     C.byref(st), _p(c), _p(h), _p(pix), _p(tiles))
    return c.reshape(n, 2), h.reshape(n, 2), pix.reshape(n, 4), tiles.reshape(n, 4)


def tile_lists(order, tiles, W, H, ts):
    """Per-tile surfel lists in depth order from per-surfel tile ranges: each surfel, in
    depth order, is appended to every tile of its range.  Returns (ranges [ntiles,2],
    flat list) with ranges as [start, end) into the flat list."""
    tx_n = (W + ts - 1) // ts
    ty_n = (H + ts - 1) // ts
    keys, vals = [], []
    tr = tiles[order]
    for r, (x0, x1, y0, y1) in enumerate(tr):
        if x0 > x1 or y0 > y1:
            continue
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                keys.append(ty * tx_n + tx)
                vals.append(order[r])
    keys = np.asarray(keys, np.int64)
    vals = np.asarray(vals, np.int64)
    perm = np.argsort(keys, kind="stable")
    keys, vals = keys[perm], vals[perm]
    ntiles = tx_n * ty_n
    starts = np.searchsorted(keys, np.arange(ntiles), side="left")
    ends = np.searchsorted(keys, np.arange(ntiles), side="right")
    return np.stack([starts, ends], axis=1), vals


def sun_camera(scene, v, S=1024):
    Bs = np.zeros(6); bs = np.zeros(2); zf = C.c_double(0)
    s = scene["surfels"]
    mean = _f32(s["mean"])
    lib().or_sun_camera(C.c_int64(mean.shape[0]), _p(mean), _p(_f32(scene["Fxy"])),
                        _p(_f32(scene.get("dF"))), _p(_f32(scene["sun"])), C.c_int32(v),
                        C.c_float(scene["b_z"]), C.c_int32(S), _p(Bs), _p(bs), C.byref(zf))
    return Bs.reshape(2, 3), bs, zf.value


def sun_depth(scene, Bs, bs, zfar, texels, settings: Settings = Settings(),
              with_ambiguity=False):
    """Sun-view depth at the given texels; with_ambiguity also returns the per-texel
    threshold-ambiguity flags of the compositing (same protocol as the main views)."""
    arrs = _surf_args(scene["surfels"])[:5]
    n = arrs[0].shape[0]
    tex = np.ascontiguousarray(texels, np.int32).reshape(-1, 2)
    out = np.zeros(tex.shape[0])
    amb = np.zeros(tex.shape[0], np.uint8)
    st = settings.c()
    lib().or_sun_depth(C.c_int64(n), *[_p(a) for a in arrs],
                       _p(np.ascontiguousarray(Bs, np.float64).ravel()),
                       _p(np.ascontiguousarray(bs, np.float64)), C.c_float(scene["b_z"]),
                       C.c_double(zfar), C.byref(st), C.c_int64(tex.shape[0]), _p(tex), _p(out),
                       _p(amb))
    return (out, amb.astype(bool)) if with_ambiguity else out


def shadow(scene, v, settings: Settings = Settings(), sel=None, with_ambiguity=False):
    """Per-surfel sun visibility of view v; with_ambiguity also returns, per surfel,
    whether any of its 3x3 sun-map texels is threshold-ambiguous."""
    arrs = _surf_args(scene["surfels"])[:5]
    n = arrs[0].shape[0]
    m = n
    if sel is not None:
        sel = np.ascontiguousarray(sel, np.int64)
        m = sel.shape[0]
    out = np.zeros(m)
    amb = np.zeros(m, np.uint8)
    st = settings.c()
    lib().or_shadow(C.c_int64(n), *[_p(a) for a in arrs], _p(_f32(scene["Fxy"])),
                    _p(_f32(scene.get("dF"))), _p(_f32(scene["sun"])), C.c_int32(v),
                    C.c_float(scene["b_z"]), C.c_int32(settings.sun_map_size), C.byref(st),
                    C.c_int64(m if sel is not None else 0), _p(sel), _p(out), _p(amb))
    return (out, amb.astype(bool)) if with_ambiguity else out


def num_threads():
    return int(lib().or_num_threads())


def set_threads(n: int):
    """Thread count of the oracle's parallel loops (timing only)."""
    lib().or_set_threads(C.c_int32(int(n)))
