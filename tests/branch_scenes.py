"""Tiny scenes that drive the rasterizer through its rarely taken branches.

Built on the seeded generator, then edited so that some surfels
  * clamp: opacity in (0.993, 0.9995) with the centre on a pixel centre of view 0 and
    the surfel lifted above the scene, so o*G exceeds alpha_max = 0.99 there (the clamp
    reading of Eq. rasterization), and the backward divides by 1 - 0.99;
  * are degenerate: the t_v axis along the viewing direction of one view (the splat is
    seen edge-on, Sec. 3.2 "Degenerate Solutions"), and, in an extra exact-nadir view,
    a vertical t_v, for which det T is exactly zero.
Used by the oracle pins (CPU) and by the GPU parity tests.
"""
import numpy as np

import synth


def _unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


def branch_scene(seed=31, n=220, views=((26, 22), (19, 24)), n_clamp=24, n_deg=16,
                 nadir_view=True):
    sc = synth.make_scene(synth.tiny(n_surfels=n, views=views, seed=seed))
    s = sc["surfels"]
    rng = np.random.default_rng(seed)
    V = len(views)
    W, H = [list(sc["width"])], [list(sc["height"])]
    Fxy, dF = sc["Fxy"], sc["dF"]
    if nadir_view:
        # exact nadir view: B = diag(1/g, -1/g) on x, y and zero on z, no camera delta
        g, w, h = 1.0, 24, 20
        F = np.array([[[1.0 / g, 0, 0, w / 2], [0, -1.0 / g, 0, h / 2]]], np.float32)
        Fxy = np.concatenate([Fxy, F])
        dF = np.concatenate([dF, np.zeros((1, 2, 4), np.float32)])
        W[0].append(w)
        H[0].append(h)
        for k in ("colC", "colc", "ambient"):
            if sc[k] is not None:
                sc[k] = np.concatenate([sc[k], sc[k][:1]])
        if sc["sun"] is not None:
            sc["sun"] = np.concatenate([sc["sun"], sc["sun"][:1]])
    sc["Fxy"], sc["dF"] = Fxy.astype(np.float32), dF.astype(np.float32)
    sc["width"] = np.asarray(W[0], np.int32)
    sc["height"] = np.asarray(H[0], np.int32)
    ztop = float(s["mean"][:, 2].max()) + 0.5
    # clamped surfels centred on pixel centres of view 0
    F0 = sc["Fxy"][0].astype(np.float64) + sc["dF"][0].astype(np.float64)
    B, b = F0[:, :3], F0[:, 3]
    for k in range(n_clamp):
        z = ztop + 0.01 * k if k % 2 == 0 else float(s["mean"][k, 2])
        x = np.array([rng.integers(2, views[0][0] - 2) + 0.5, rng.integers(2, views[0][1] - 2) + 0.5])
        xy = np.linalg.solve(B[:, :2], x - b - B[:, 2] * z)
        s["mean"][k] = np.array([xy[0], xy[1], z], np.float32)
        s["opacity"][k] = np.float32(rng.uniform(0.993, 0.9995))
        s["scale"][k] = np.float32(rng.uniform(1.0, 2.0, size=2))
    # surfels seen edge-on: t_v along the viewing direction d = B_x x B_y of a view
    k0 = n_clamp
    for i in range(n_deg):
        k = k0 + i
        v = i % V
        Fv = sc["Fxy"][v].astype(np.float64) + sc["dF"][v].astype(np.float64)
        d = _unit(np.cross(Fv[0, :3], Fv[1, :3]))
        tu = _unit(np.cross(d, rng.normal(size=3)))
        s["t_v"][k] = d.astype(np.float32)
        s["t_u"][k] = tu.astype(np.float32)
        s["opacity"][k] = np.float32(rng.uniform(0.4, 0.95))
    if nadir_view:
        # vertical t_v: exactly degenerate in the nadir view (T's second column is 0)
        for i in range(n_deg // 2):
            k = k0 + n_deg + i
            s["t_v"][k] = np.array([0, 0, 1], np.float32)
            s["t_u"][k] = _unit([1.0, rng.normal(), 0.0]).astype(np.float32)
            s["opacity"][k] = np.float32(rng.uniform(0.4, 0.95))
    return sc


def special_surfels(sc, n_clamp=24, n_deg=16, nadir_view=True):
    """Indices of the clamped and degenerate surfels of branch_scene."""
    extra = n_deg // 2 if nadir_view else 0
    return np.arange(0, n_clamp), np.arange(n_clamp, n_clamp + n_deg + extra)
