"""Ground truth for the geometric shadow pass (Sec. 3.1 shadow-mapping note, Sec. 3.3 sun
camera, Supp. A): sun visibility of points on a DSM heightfield by marching the ray
towards the sun over the heightfield itself, independent of surfels and shadow maps.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke entry point and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path.

Geometry: the sun at azimuth phi (from +x towards +y) and elevation theta lies along
s = (cos phi / tan theta, sin phi / tan theta, 1); a point q at altitude z_q is in shadow
when some point of the ray q + t s (t > 0) lies below the surface, i.e. when the height
H(x, y) of the DSM (bilinear between its nodes) exceeds z_q + L tan theta at horizontal
distance L along (cos phi, sin phi).  `sun_margin` returns the largest such excess over
the march; its sign decides, and its size is how far (in metres of altitude) the decision
is from changing.
"""
from __future__ import annotations

import math

import numpy as np


def bilinear(coords, z, x, y):
    """Height of the DSM (nodes z[j, i] at (coords[i], coords[j]), square grid) at (x, y);
    NaN outside the grid."""
    z = np.asarray(z, np.float64)
    g = float(coords[1] - coords[0])
    n_y, n_x = z.shape
    fi = (np.asarray(x, np.float64) - coords[0]) / g
    fj = (np.asarray(y, np.float64) - coords[0]) / g
    inside = (fi >= 0) & (fi <= n_x - 1) & (fj >= 0) & (fj <= n_y - 1)
    i = np.clip(np.floor(fi).astype(np.int64), 0, n_x - 2)
    j = np.clip(np.floor(fj).astype(np.int64), 0, n_y - 2)
    fx = np.clip(fi - i, 0.0, 1.0)
    fy = np.clip(fj - j, 0.0, 1.0)
    h = (z[j, i] * (1 - fx) + z[j, i + 1] * fx) * (1 - fy) + \
        (z[j + 1, i] * (1 - fx) + z[j + 1, i + 1] * fx) * fy
    return np.where(inside, h, np.nan)


def window_filter(z, r, reduce):
    """Max (reduce=np.maximum) or min (np.minimum) of the DSM over the (2r+1)^2 nodes
    around each node (clipped at the grid's border): a heightfield grown (or shrunk)
    sideways by r nodes, to mark points whose decision could change if the surface
    moved sideways that far."""
    z = np.asarray(z, np.float64)
    out = z.copy()
    n0, n1 = z.shape
    for dj in range(-r, r + 1):
        for di in range(-r, r + 1):
            dst = (slice(max(0, dj), n0 + min(0, dj)), slice(max(0, di), n1 + min(0, di)))
            src = (slice(max(0, -dj), n0 + min(0, -dj)), slice(max(0, -di), n1 + min(0, -di)))
            out[dst] = reduce(out[dst], z[src])
    return out


def sun_margin(coords, z, points, phi, theta, start=0.0, step=None):
    """max over L in [start, L_max] of H(q + L u) - (z_q + L tan theta) for every point q
    (rows of `points`, metres); u = (cos phi, sin phi).  The march starts `start` metres
    from the point (excluding its own neighbourhood), steps a quarter grid spacing (or
    `step`), and ends where the ray has risen above the highest node.  Positive: shadowed;
    negative: lit.  Points whose ray leaves the grid at once get -inf."""
    p = np.asarray(points, np.float64).reshape(-1, 3)
    g = float(coords[1] - coords[0])
    step = g / 4 if step is None else float(step)
    tn = math.tan(theta)
    ux, uy = math.cos(phi), math.sin(phi)
    L_max = (float(np.max(z)) - p[:, 2].min()) / tn + g if p.shape[0] else 0.0
    best = np.full(p.shape[0], -np.inf)
    L = start if start > 0 else step
    while L <= L_max + step:
        h = bilinear(coords, z, p[:, 0] + L * ux, p[:, 1] + L * uy)
        excess = h - (p[:, 2] + L * tn)
        best = np.where(np.isnan(excess), best, np.maximum(best, excess))
        L += step
    return best
