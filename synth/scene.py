"""Seeded synthetic satellite scenes: DSM, surfels, affine cameras, suns, colour terms.

This module builds *inputs* only. It holds none of the rasterizer's arithmetic (no
projection, compositing, sun camera or shadow test), so that both the FP64 oracle and
the HIP path can consume the same arrays without sharing any of the method's code.

Recipe (each step follows the paper's description of its data and initialisation):
  * DSM on a regular grid at 0.5 m GSD, centred at the origin: flat ground (optionally
    with a 3-octave gradient-noise relief, written here from Perlin's published
    gradient-noise construction) plus axis-aligned boxes.  The paper's sites are
    ~256 m tiles at 0.3-0.5 m GSD (Sec. 4, experimental setup); the stand-in scenes keep
    the GSD and vary the extent.
  * Surfel centres by area-weighted sampling of DSM cells, a = |dx x dy| from finite
    differences (Sec. 3.4, "Area-Weighted Sampling"), jittered inside the cell on the
    bilinear surface.
  * Frames from the local DSM normal tilted by N(0, 5 deg), tangent axes by Gram-Schmidt
    of a random vector (Sec. 3.4, "Splat Orientation").
  * Scales log-uniform in [0.2, 2] m, opacity sigmoid(N(0,1)), albedo U[0,1]^3 (the
    shadow ground-truth scenes use small opaque surfels instead: `shadow_city`).
  * Affine cameras from off-nadir / azimuth with a small random affine distortion of the
    image axes, mapping world metres to pixels (Sec. 3.1, "Affine camera model").
  * Camera deltas, colour gain/bias, ambient light and sun angles as the configurations
    state.
Everything is drawn from numpy PCG64 streams spawned from one master seed in a fixed
order: scene, surfels, cameras, suns, delta-F, colour, upstream gradients.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

STREAMS = ("scene", "surfels", "cameras", "suns", "dF", "colour", "grads")


@dataclasses.dataclass
class SceneSpec:
    """Parameters of one synthetic workload."""
    name: str
    extent: float                   # scene side in metres (square, centred at origin)
    n_boxes: int
    box_side: Tuple[float, float]   # footprint side range, metres
    box_height: Tuple[float, float] # height range, metres
    relief: float                   # max amplitude of the ground relief, metres (0 = flat)
    n_surfels: int
    view_sizes: List[Tuple[int, int]]  # (width, height) per view
    off_nadir: Tuple[float, float] = (5.0, 30.0)  # degrees
    dF_rel: float = 0.0             # camera-delta std, relative to |F_ij|
    colour: bool = False            # non-identity colour correction + ambient
    suns: bool = False              # per-view sun (azimuth, elevation)
    sun_elev: Tuple[float, float] = (30.0, 70.0)
    gsd: float = 0.5                # DSM grid spacing, metres
    fill: float = 0.95              # fraction of the image the scene box fills
    seed: int = 0
    scale_range: Tuple[float, float] = (0.2, 2.0)  # surfel scales, log-uniform, metres
    opacity: Optional[float] = None  # fixed opacity (None: sigmoid(N(0, 1)))
    tilt_deg: float = 5.0           # std of the normal's tilt from the DSM normal


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    children = ss.spawn(len(STREAMS))
    return {k: np.random.Generator(np.random.PCG64(c)) for k, c in zip(STREAMS, children)}


# ----------------------------------------------------------------------------- DSM
def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def gradient_noise(x, y, wavelength, rng):
    """2D gradient noise (Perlin): random unit gradients on an integer lattice,
    quintic fade, bilinear blend of the four corner dot products."""
    gx = x / wavelength
    gy = y / wavelength
    x0 = np.floor(gx).astype(np.int64)
    y0 = np.floor(gy).astype(np.int64)
    xmin, ymin = int(x0.min()), int(y0.min())
    nx, ny = int(x0.max()) - xmin + 2, int(y0.max()) - ymin + 2
    ang = rng.uniform(0.0, 2.0 * np.pi, size=(ny, nx))
    gvx, gvy = np.cos(ang), np.sin(ang)
    fx, fy = gx - x0, gy - y0
    ix, iy = x0 - xmin, y0 - ymin

    def corner(dx, dy):
        vx = gvx[iy + dy, ix + dx]
        vy = gvy[iy + dy, ix + dx]
        return vx * (fx - dx) + vy * (fy - dy)

    u, v = _fade(fx), _fade(fy)
    n00, n10, n01, n11 = corner(0, 0), corner(1, 0), corner(0, 1), corner(1, 1)
    return (n00 * (1 - u) + n10 * u) * (1 - v) + (n01 * (1 - u) + n11 * u) * v


def make_dsm(spec: SceneSpec, rng):
    """Node heights z[j, i] at x = -E/2 + i*g, y = -E/2 + j*g."""
    n = int(round(spec.extent / spec.gsd)) + 1
    coords = -spec.extent / 2 + spec.gsd * np.arange(n)
    X, Y = np.meshgrid(coords, coords)
    z = np.zeros((n, n), dtype=np.float64)
    if spec.relief > 0:
        rel = np.zeros_like(z)
        for octave in range(3):
            rel += (0.5 ** octave) * gradient_noise(X, Y, 200.0 / (2 ** octave), rng)
        m = np.abs(rel).max()
        if m > 0:
            rel *= spec.relief / m
        z += rel
    for _ in range(spec.n_boxes):
        sx, sy = rng.uniform(*spec.box_side, size=2)
        h = rng.uniform(*spec.box_height)
        cx, cy = rng.uniform(-spec.extent / 2, spec.extent / 2, size=2)
        i0 = int(np.searchsorted(coords, cx - sx / 2))
        i1 = int(np.searchsorted(coords, cx + sx / 2))
        j0 = int(np.searchsorted(coords, cy - sy / 2))
        j1 = int(np.searchsorted(coords, cy + sy / 2))
        if i1 > i0 and j1 > j0:
            blk = z[j0:j1, i0:i1]
            base = float(blk.min())
            np.maximum(blk, base + h, out=blk)
    return coords, z


# -------------------------------------------------------------------------- surfels
def _rotate(v, axis, ang):
    """Rodrigues rotation of row vectors v about unit row axes by angles ang."""
    c, s = np.cos(ang)[:, None], np.sin(ang)[:, None]
    return v * c + np.cross(axis, v) * s + axis * np.sum(axis * v, axis=1, keepdims=True) * (1 - c)


def _unit(v):
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def sample_surfels(spec: SceneSpec, coords, z, rng):
    g = spec.gsd
    z00, z10 = z[:-1, :-1], z[:-1, 1:]
    z01, z11 = z[1:, :-1], z[1:, 1:]
    dzdx = 0.5 * ((z10 - z00) + (z11 - z01)) / g
    dzdy = 0.5 * ((z01 - z00) + (z11 - z10)) / g
    # |dx x dy| with dx = (g, 0, g dzdx), dy = (0, g, g dzdy)
    area = g * g * np.sqrt(dzdx ** 2 + dzdy ** 2 + 1.0)
    p = (area / area.sum()).ravel()
    n = spec.n_surfels
    cell = rng.choice(p.size, size=n, p=p)
    cj, ci = np.divmod(cell, z00.shape[1])
    fx = rng.uniform(0.0, 1.0, size=n)
    fy = rng.uniform(0.0, 1.0, size=n)
    a00, a10, a01, a11 = z00[cj, ci], z10[cj, ci], z01[cj, ci], z11[cj, ci]
    zz = (a00 * (1 - fx) + a10 * fx) * (1 - fy) + (a01 * (1 - fx) + a11 * fx) * fy
    gx = ((1 - fy) * (a10 - a00) + fy * (a11 - a01)) / g
    gy = ((1 - fx) * (a01 - a00) + fx * (a11 - a10)) / g
    mean = np.stack([coords[ci] + fx * g, coords[cj] + fy * g, zz], axis=1)
    normal = _unit(np.stack([-gx, -gy, np.ones(n)], axis=1))
    # tilt by N(0, 5 deg) about a random tangent axis
    r = rng.normal(size=(n, 3))
    axis = _unit(r - np.sum(r * normal, axis=1, keepdims=True) * normal)
    normal = _unit(_rotate(normal, axis, np.deg2rad(rng.normal(0.0, spec.tilt_deg, size=n))))
    # Gram-Schmidt frame
    r = rng.normal(size=(n, 3))
    t_u = _unit(r - np.sum(r * normal, axis=1, keepdims=True) * normal)
    t_v = np.cross(normal, t_u)
    lo, hi = spec.scale_range
    scale = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(n, 2)))
    opacity = 1.0 / (1.0 + np.exp(-rng.normal(size=n)))
    if spec.opacity is not None:
        opacity = np.full(n, spec.opacity)
    albedo = rng.uniform(0.0, 1.0, size=(n, 3))
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return dict(mean=f32(mean), t_u=f32(t_u), t_v=f32(t_v), scale=f32(scale),
                opacity=f32(opacity), albedo=f32(albedo))


# -------------------------------------------------------------------------- cameras
def affine_camera(off_nadir_deg, azimuth_deg, width, height, box_lo, box_hi, rng,
                  fill=0.95, skew=0.01):
    """World metres -> pixel affine camera F_xy (2x4), looking along
    d = (sin nu cos psi, sin nu sin psi, -cos nu), image axes perpendicular to d,
    a small random affine distortion, scaled so the scene box fills `fill` of the image."""
    nu, psi = np.deg2rad(off_nadir_deg), np.deg2rad(azimuth_deg)
    d = np.array([np.sin(nu) * np.cos(psi), np.sin(nu) * np.sin(psi), -np.cos(nu)])
    e1 = np.array([1.0, 0.0, 0.0]) - d[0] * d
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d, e1)
    A = np.eye(2) + rng.normal(0.0, skew, size=(2, 2))
    B = A @ np.stack([e1, e2])
    corners = np.array([[x, y, zc] for x in (box_lo[0], box_hi[0])
                        for y in (box_lo[1], box_hi[1]) for zc in (box_lo[2], box_hi[2])])
    proj = corners @ B.T
    lo, hi = proj.min(axis=0), proj.max(axis=0)
    gsd = max((hi[0] - lo[0]) / (fill * width), (hi[1] - lo[1]) / (fill * height))
    B = B / gsd
    mid = 0.5 * (lo + hi) / gsd
    b = np.array([width / 2.0, height / 2.0]) - mid
    return np.concatenate([B, b[:, None]], axis=1)


def make_scene(spec: SceneSpec):
    rs = _streams(spec.seed)
    coords, z = make_dsm(spec, rs["scene"])
    surf = sample_surfels(spec, coords, z, rs["surfels"])
    zmax = float(z.max())
    b_z = np.float32(zmax + 10.0)
    lo = np.array([-spec.extent / 2, -spec.extent / 2, float(z.min())])
    hi = np.array([spec.extent / 2, spec.extent / 2, zmax])
    V = len(spec.view_sizes)
    width = np.array([w for w, _ in spec.view_sizes], dtype=np.int32)
    height = np.array([h for _, h in spec.view_sizes], dtype=np.int32)
    Fxy = np.zeros((V, 2, 4))
    for v in range(V):
        nu = rs["cameras"].uniform(*spec.off_nadir)
        psi = rs["cameras"].uniform(0.0, 360.0)
        Fxy[v] = affine_camera(nu, psi, width[v], height[v], lo, hi, rs["cameras"], spec.fill)
    Fxy = Fxy.astype(np.float32)
    dF = np.zeros((V, 2, 4), dtype=np.float32)
    if spec.dF_rel > 0:
        dF = (spec.dF_rel * np.abs(Fxy) * rs["dF"].normal(size=(V, 2, 4))).astype(np.float32)
    if spec.colour:
        colC = (np.eye(3)[None] + rs["colour"].normal(0.0, 0.05, size=(V, 3, 3))).astype(np.float32)
        colc = rs["colour"].normal(0.0, 0.02, size=(V, 3)).astype(np.float32)
        amb = rs["colour"].uniform(0.1, 0.4, size=(V, 3)).astype(np.float32)
    else:
        colC = colc = amb = None
    sun = None
    if spec.suns:
        phi = rs["suns"].uniform(0.0, 2 * np.pi, size=V)
        theta = np.deg2rad(rs["suns"].uniform(*spec.sun_elev, size=V))
        sun = np.stack([phi, theta], axis=1).astype(np.float32)
    return dict(spec=spec, surfels=surf, width=width, height=height, Fxy=Fxy, dF=dF,
                colC=colC, colc=colc, ambient=amb, sun=sun, b_z=float(b_z),
                dsm=(coords, z))


def pixel_offsets(width, height):
    sizes = np.asarray(width, np.int64) * np.asarray(height, np.int64)
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def upstream_grads(scene, seed_offset=0):
    """Seeded N(0,1) upstream gradients for image (3 ch), depth (1) and normal (3),
    planar CHW per view, concatenated over views."""
    rs = _streams(scene["spec"].seed + seed_offset)["grads"]
    P = int(pixel_offsets(scene["width"], scene["height"])[-1])
    dI = rs.standard_normal(3 * P, dtype=np.float32)
    dD = rs.standard_normal(P, dtype=np.float32)
    dN = rs.standard_normal(3 * P, dtype=np.float32)
    return dI, dD, dN


# ---------------------------------------------------------------------- workloads
def config(k: int, views: Optional[Sequence[Tuple[int, int]]] = None) -> SceneSpec:
    """The five stated workloads (k = 1..5); master seed 1000 + k."""
    if k == 1:
        return SceneSpec("c1_tiny_20k_256px", 128.0, 10, (8.0, 30.0), (3.0, 30.0), 0.0,
                         20_000, list(views or [(256, 256)]), seed=1001)
    if k == 2:
        return SceneSpec("c2_1M_2048px", 1000.0, 500, (10.0, 40.0), (3.0, 80.0), 2.0,
                         1_000_000, list(views or [(2048, 2048)]), dF_rel=1e-3,
                         colour=True, seed=1002)
    if k == 3:
        if views is None:
            r = np.random.Generator(np.random.PCG64(np.random.SeedSequence(1003).spawn(8)[7]))
            views = [(int(r.integers(1024, 2049)), int(r.integers(1024, 2049))) for _ in range(40)]
        return SceneSpec("c3_2M_40views", 1000.0, 500, (10.0, 40.0), (3.0, 80.0), 2.0,
                         2_000_000, list(views), off_nadir=(5.0, 35.0), dF_rel=1e-3,
                         colour=True, suns=True, seed=1003)
    if k == 5:
        return SceneSpec("c5_5M_50views", 2000.0, 2000, (10.0, 40.0), (3.0, 80.0), 2.0,
                         5_000_000, list(views or [(2048, 2048)] * 50), off_nadir=(5.0, 35.0),
                         dF_rel=1e-3, colour=True, suns=True, seed=1005)
    raise ValueError(f"no scene config {k}")


def tiny(n_surfels=48, views=((40, 33),), extent=24.0, n_boxes=2, seed=7, colour=True,
         suns=True, dF_rel=1e-3, box_height=(2.0, 6.0), box_side=(4.0, 8.0), gsd=0.5):
    """Small scenes for oracle pins and parity tests (ragged, not tile multiples)."""
    return SceneSpec(f"tiny_{n_surfels}", extent, n_boxes, box_side, box_height, 0.0,
                     n_surfels, list(views), dF_rel=dF_rel, colour=colour, suns=suns,
                     seed=seed, gsd=gsd)


def shadow_city(n_surfels=30_000, extent=48.0, n_boxes=6, views=3, seed=5):
    """A city whose surfels follow the DSM closely (0.3 m, opacity 0.95, no tilt), so that
    the DSM heightfield is the ground truth of its shadows; one 64^2 nadir-ish view per
    sun (the views only carry the suns)."""
    return SceneSpec(f"shadow_city_{n_surfels}", extent, n_boxes, (6.0, 14.0), (3.0, 12.0), 0.0,
                     n_surfels, [(64, 64)] * views, suns=True, seed=seed,
                     scale_range=(0.3, 0.3), opacity=0.95, tilt_deg=0.0)
