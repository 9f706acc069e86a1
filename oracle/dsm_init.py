"""FP64 oracle of the geometry-aware initialisation (Sec. 3.4): area-weighted sampling of
surfel centres on a DSM and their orientation from the local surface normal.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke entry point and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path; the random
numbers come from Philox4x32-10 (Salmon et al., "Parallel random numbers: as easy as 1, 2,
3", SC 2011), implemented here from its published definition (the HIP path has its own).

Readings (the paper gives the weight a = |dx x dy| from finite differences, the
normalised sampling distribution and the Gram-Schmidt frame; the rest is fixed here):
* the DSM is a grid of node heights z[j, i] at (x0 + i g, y0 + j g); cell (j, i) spans
  nodes j..j+1, i..i+1; its tangents are dx = (g, 0, dzx), dy = (0, g, dzy) with dzx, dzy
  the means of the cell's two edge differences along x and y; a = g sqrt(dzx^2 + dzy^2 +
  g^2), the cell normal is (-dzx, -dzy, g) / sqrt(...);
* the sampling weights are integers, w = floor(65536 a / g^2 + 1/2) (a flat cell weighs
  2^16), so every sampling decision is exact; cumulative weights in row-major cell order;
* sample k draws Philox4x32-10 with key (seed low, seed high) at counters (k, 0, 0, 0)
  -> r0..r3 and (k, 1, 0, 0) -> r4..r7: target t = (r1 2^32 + r0) mod W (W the total
  weight), cell = the first with cumulative weight > t; fractional position (r2, r3) /
  2^32 inside the cell, height bilinear in the cell's four nodes; random vector
  (r4, r5, r6) / 2^31 - 1; t_u = normalise(r - (r . n) n) (x axis if that is shorter
  than 1e-6), t_v = n x t_u;
* scale s_u = s_v = sqrt(surface area / N), surface area W g^2 / 65536; opacity and
  albedo are given constants (the paper does not state its initial values).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF
WEIGHT_ONE = 65536


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32 with 10 rounds; arguments are uint32 arrays (or scalars)."""
    c0, c1, c2, c3 = [np.asarray(x, np.uint64) & MASK for x in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, np.uint64) & MASK
    k1 = np.asarray(k1, np.uint64) & MASK
    for r in range(10):
        p0 = c0 * np.uint64(M0)
        p1 = c2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return c0, c1, c2, c3


def cell_geometry(z, g):
    """Per cell: weight (int64), area, unit normal [nc, 3], and the edge slopes."""
    z = np.asarray(z, np.float32).astype(np.float64)
    g = float(np.float32(g))
    z00, z10, z01, z11 = z[:-1, :-1], z[:-1, 1:], z[1:, :-1], z[1:, 1:]
    dzx = 0.5 * ((z10 - z00) + (z11 - z01))
    dzy = 0.5 * ((z01 - z00) + (z11 - z10))
    s = np.sqrt(dzx * dzx + dzy * dzy + g * g)
    area = g * s
    w = np.floor(area / (g * g) * WEIGHT_ONE + 0.5).astype(np.int64)
    n = np.stack([-dzx / s, -dzy / s, g / s], -1)
    return w.reshape(-1), area.reshape(-1), n.reshape(-1, 3)


def dsm_init(z, x0, y0, g, n, seed, opacity=0.5, albedo=0.5, sel=None):
    """Initial surfels (mean, t_u, t_v, scale, opacity, albedo, cell) for samples
    `sel` (default all 0..n-1)."""
    z = np.asarray(z, np.float32).astype(np.float64)
    ny, nx = z.shape
    g = float(np.float32(g))
    x0, y0 = float(np.float32(x0)), float(np.float32(y0))
    w, _, normals = cell_geometry(z, g)
    cdf = np.cumsum(w.astype(np.uint64))
    total = int(cdf[-1])
    k = np.arange(n, dtype=np.uint64) if sel is None else np.asarray(sel, np.uint64)
    key0, key1 = np.uint64(seed & MASK), np.uint64((seed >> 32) & MASK)
    zero = np.zeros_like(k)
    r0, r1, r2, r3 = philox4x32_10(k, zero, zero, zero, key0, key1)
    r4, r5, r6, _ = philox4x32_10(k, zero + np.uint64(1), zero, zero, key0, key1)
    t = ((r1 << np.uint64(32)) | r0) % np.uint64(total)
    cell = np.searchsorted(cdf, t, side="right")
    cj, ci = np.divmod(cell, nx - 1)
    fx = r2.astype(np.float64) / 2.0 ** 32
    fy = r3.astype(np.float64) / 2.0 ** 32
    a00, a10, a01, a11 = z[cj, ci], z[cj, ci + 1], z[cj + 1, ci], z[cj + 1, ci + 1]
    zz = (a00 * (1 - fx) + a10 * fx) * (1 - fy) + (a01 * (1 - fx) + a11 * fx) * fy
    mean = np.stack([x0 + (ci + fx) * g, y0 + (cj + fy) * g, zz], 1)
    nrm = normals[cell]
    rv = np.stack([r4, r5, r6], 1).astype(np.float64) / 2.0 ** 31 - 1.0
    u = rv - np.sum(rv * nrm, 1, keepdims=True) * nrm
    un = np.linalg.norm(u, axis=1, keepdims=True)
    xa = np.array([1.0, 0.0, 0.0])
    bad = un[:, 0] < 1e-6
    u[bad] = xa - nrm[bad] * (nrm[bad] @ xa)[:, None]
    un = np.linalg.norm(u, axis=1, keepdims=True)
    t_u = u / un
    t_v = np.cross(nrm, t_u)
    spacing = np.sqrt(total * g * g / WEIGHT_ONE / n)
    m = k.size
    return dict(mean=mean, t_u=t_u, t_v=t_v, scale=np.full((m, 2), spacing),
                opacity=np.full(m, float(np.float32(opacity))), albedo=np.full((m, 3), float(np.float32(albedo))),
                cell=cell.astype(np.int64), normal=nrm, total_weight=total)
