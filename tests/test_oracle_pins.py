"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage of SatSplat (arXiv 2606.28581) it pins.  None of them
re-types the oracle's own formula: expected values come from closed forms written in a
different way (covariance form of the Gaussian, line-plane intersection, telescoping
sums), invariants, finite differences, or brute force on tiny inputs.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import Settings

ST = Settings()


def F32(x):
    """Inputs reach the oracle as FP32; expected values use the same rounded inputs."""
    return np.asarray(x, np.float32).astype(np.float64)


def custom_scene(surfels, views, bz=50.0, dF=None, colC=None, colc=None, amb=None, sun=None):
    """surfels: list of dicts with p, tu, tv, s (2), o, a (3); views: list of (W,H,F[2,4])."""
    f = lambda k, d: np.asarray([x[k] for x in surfels], np.float32).reshape(len(surfels), d)
    surf = dict(mean=f("p", 3), t_u=f("tu", 3), t_v=f("tv", 3), scale=f("s", 2),
                opacity=f("o", 1).reshape(-1), albedo=f("a", 3))
    V = len(views)
    return dict(surfels=surf, width=np.array([v[0] for v in views], np.int32),
                height=np.array([v[1] for v in views], np.int32),
                Fxy=np.asarray([v[2] for v in views], np.float32),
                dF=np.zeros((V, 2, 4), np.float32) if dF is None else np.asarray(dF, np.float32),
                colC=colC, colc=colc, ambient=amb, sun=sun, b_z=float(np.float32(bz)))


def nadir(g, W, H, cx=0.0, cy=0.0):
    return [[1.0 / g, 0, 0, W / 2 - cx / g], [0, -1.0 / g, 0, H / 2 + cy / g]]


def planar(out, key, W, H, ch):
    return out[key].reshape(ch, H, W) if ch > 1 else out[key].reshape(H, W)


def pixel_centres(W, H):
    ys, xs = np.meshgrid(np.arange(H) + 0.5, np.arange(W) + 0.5, indexing="ij")
    return xs, ys


# ---------------------------------------------------------------- P1 analytic Gaussian
@pytest.mark.parametrize("o", [0.8, 0.995, 0.999])
def test_p1_horizontal_surfel_nadir_camera_is_analytic_gaussian(o):
    """Sec. 3.2 Eqs. affine2dgs_screen2uv / affine2dgs_Qq + depth function: a horizontal
    surfel under a nadir camera renders an axis-aligned Gaussian of std s/g pixels,
    alpha = min(0.99, o exp(-rho/2)).  With o > 0.99 the clamp is active near the centre
    (alpha_max reading of Eq. rasterization)."""
    g, W, H = 0.5, 48, 40
    su, sv, a, pz = 3.0, 1.7, (0.3, 0.6, 0.9), 4.0
    sc = custom_scene([dict(p=(1.3, -0.7, pz), tu=(1, 0, 0), tv=(0, 1, 0), s=(su, sv), o=o, a=a)],
                      [(W, H, nadir(g, W, H))], bz=50.0)
    out = oracle.forward(sc, ST)
    xs, ys = pixel_centres(W, H)
    su, sv, o, a, pz = [F32(x) for x in (su, sv, o, a, pz)]
    cx, cy = W / 2 + F32(1.3) / g, H / 2 + F32(0.7) / g
    rho = ((xs - cx) * g / su) ** 2 + ((ys - cy) * g / sv) ** 2
    alpha = np.minimum(F32(0.99), o * np.exp(-0.5 * rho))
    alpha = np.where(alpha >= ST.alpha_min, alpha, 0.0)
    clamped = o * np.exp(-0.5 * rho) > F32(0.99)
    assert clamped.any() == (o > F32(0.99))
    A = planar(out, "albedo", W, H, 3)
    for ch in range(3):
        np.testing.assert_allclose(A[ch], a[ch] * alpha, atol=1e-12)
    np.testing.assert_allclose(planar(out, "depth", W, H, 1), alpha * (np.float32(50.0) - pz),
                               atol=1e-10)
    N = planar(out, "normal", W, H, 3)
    np.testing.assert_allclose(N[2], alpha, atol=1e-12)
    np.testing.assert_allclose(N[:2], 0.0, atol=1e-12)
    np.testing.assert_allclose(planar(out, "T", W, H, 1), 1.0 - alpha, atol=1e-12)


def test_p1_oblique_camera_tilted_surfel_has_covariance_TTt():
    """Under any affine camera the splat is a 2D Gaussian with covariance T T^T, T = B_xy RS'
    (Sec. 3.2): rho = delta^T (T T^T)^-1 delta, written here via a linear solve."""
    rng = np.random.default_rng(3)
    W, H = 40, 36
    F = np.array([[1.7, 0.4, -0.3, 20.0], [0.2, -1.9, 0.5, 18.0]])
    n = np.array([0.3, -0.2, 1.0]); n /= np.linalg.norm(n)
    tu = np.cross(n, [0.0, 1.0, 0.0]); tu /= np.linalg.norm(tu)
    tv = np.cross(n, tu)
    p, s, o = np.array([0.5, -0.4, 2.0]), np.array([2.5, 1.2]), 0.7
    sc = custom_scene([dict(p=p, tu=tu, tv=tv, s=s, o=o, a=(1, 1, 1))], [(W, H, F)])
    st = Settings(lowpass_mode=1)   # plain Gaussian, no low-pass floor
    out = oracle.forward(sc, st)
    f64 = lambda x: np.asarray(np.float32(x), np.float64)
    B, b = f64(F)[:, :3], f64(F)[:, 3]
    M = np.stack([f64(s[0]) * f64(tu), f64(s[1]) * f64(tv)], axis=1)
    T = B @ M
    c = B @ f64(p) + b
    xs, ys = pixel_centres(W, H)
    d = np.stack([xs - c[0], ys - c[1]], -1).reshape(-1, 2)
    rho = np.sum(d * np.linalg.solve(T @ T.T, d.T).T, axis=1).reshape(H, W)
    alpha = np.minimum(np.float32(0.99), f64(o) * np.exp(-0.5 * rho))
    alpha = np.where(alpha >= ST.alpha_min, alpha, 0.0)
    np.testing.assert_allclose(planar(out, "albedo", W, H, 3)[0], alpha, atol=1e-12)
    assert (alpha > 0).sum() > 50


# ---------------------------------------------------------------- P2 low-pass floor
@pytest.mark.parametrize("mode", [0, 1])
def test_p2_subpixel_and_degenerate_surfels_render_lowpass_disk(mode):
    """Sec. 3.2 'Degenerate Solutions': the lower-bounded Gaussian G((x-c)/sigma) is what
    a sub-pixel or edge-on splat shows: exp(-|x-c|^2 / (2 sigma^2)) * o."""
    g, W, H = 0.5, 20, 20
    surf = []
    if mode == 0:   # sub-pixel (s/g = 0.1 << sigma) only floors in mode 0
        surf.append(dict(p=(0.2, 0.1, 1.0), tu=(1, 0, 0), tv=(0, 1, 0), s=(0.05, 0.05), o=0.9, a=(1, 1, 1)))
    else:           # edge-on under a nadir camera: t_v along z, det(T) = 0
        surf.append(dict(p=(0.2, 0.1, 1.0), tu=(1, 0, 0), tv=(0, 0, 1), s=(2.0, 2.0), o=0.9, a=(1, 1, 1)))
    sc = custom_scene(surf, [(W, H, nadir(g, W, H))])
    out = oracle.forward(sc, Settings(lowpass_mode=mode))
    xs, ys = pixel_centres(W, H)
    cx, cy = W / 2 + F32(0.2) / g, H / 2 - F32(0.1) / g
    sig = np.float64(np.float32(0.70710678))
    alpha = np.minimum(np.float32(0.99), np.float64(np.float32(0.9)) *
                       np.exp(-((xs - cx) ** 2 + (ys - cy) ** 2) / (2 * sig * sig)))
    alpha = np.where(alpha >= ST.alpha_min, alpha, 0.0)
    np.testing.assert_allclose(planar(out, "albedo", W, H, 3)[1], alpha, atol=1e-12)


# ---------------------------------------------------------------- P3 telescoping
def test_p3_weights_plus_final_transmittance_is_one():
    """Eq. rasterization: sum_i alpha_i prod_{j<i}(1-alpha_j) + prod_i (1-alpha_i) = 1."""
    sc = synth.make_scene(synth.tiny(n_surfels=400, views=((37, 29), (20, 45))))
    sc["surfels"]["albedo"][:] = 1.0
    sc["colC"] = sc["colc"] = sc["ambient"] = None
    out = oracle.forward(sc, ST)
    P = out["T"].shape[0]
    A = np.concatenate([out["albedo"][3 * o:3 * o + 3 * p].reshape(3, p)
                        for o, p in [(0, 37 * 29), (37 * 29, 20 * 45)]], axis=1)
    for ch in range(3):
        np.testing.assert_allclose(A[ch] + out["T"], 1.0, atol=1e-13)
    assert (out["T"] < 0.5).mean() > 0.3 and P == 37 * 29 + 20 * 45


# ---------------------------------------------------------------- P4 compositing order
def test_p4_stacked_surfels_closed_form_and_input_order_invariance():
    """Eq. rasterization with index i ordered by depth (Sec. 3.2): three stacked discs give
    f1 a1 + f2 a2 (1-a1) + f3 a3 (1-a1)(1-a2), whatever order the input lists them in."""
    g, W, H = 0.5, 16, 16
    surf = [dict(p=(0, 0, z), tu=(1, 0, 0), tv=(0, 1, 0), s=(2.0, 2.0), o=o, a=a)
            for z, o, a in [(3.0, 0.4, (1, 0, 0)), (7.0, 0.3, (0, 1, 0)), (5.0, 0.5, (0, 0, 1))]]
    sc = custom_scene(surf, [(W, H, nadir(g, W, H))])
    out = oracle.forward(sc, ST)
    xs, ys = pixel_centres(W, H)
    G = np.exp(-0.5 * (((xs - 8) * g / 2.0) ** 2 + ((ys - 8) * g / 2.0) ** 2))
    f32 = lambda x: np.float64(np.float32(x))
    a_top, a_mid, a_low = f32(0.3) * G, f32(0.5) * G, f32(0.4) * G   # z = 7, 5, 3
    A = planar(out, "albedo", W, H, 3)
    np.testing.assert_allclose(A[1], a_top, atol=1e-12)
    np.testing.assert_allclose(A[2], a_mid * (1 - a_top), atol=1e-12)
    np.testing.assert_allclose(A[0], a_low * (1 - a_top) * (1 - a_mid), atol=1e-12)
    sc2 = custom_scene([surf[2], surf[0], surf[1]], [(W, H, nadir(g, W, H))])
    out2 = oracle.forward(sc2, ST)
    np.testing.assert_array_equal(out2["albedo"], out["albedo"])


def test_p4_random_permutation_with_distinct_keys_is_invariant():
    sc = synth.make_scene(synth.tiny(n_surfels=300, views=((33, 27),)))
    sc["surfels"]["mean"][:, 2] += np.arange(300, dtype=np.float32) * np.float32(1e-3)
    kap = np.float32(sc["b_z"]) - sc["surfels"]["mean"][:, 2]
    assert np.unique(kap).size == kap.size
    out = oracle.forward(sc, ST)
    perm = np.random.default_rng(0).permutation(300)
    sc2 = dict(sc, surfels={k: v[perm] for k, v in sc["surfels"].items()})
    out2 = oracle.forward(sc2, ST)
    for k in ("image", "depth", "normal", "T"):
        np.testing.assert_allclose(out2[k], out[k], atol=1e-13)


def test_depth_order_is_sorted_fp32_key_with_index_ties():
    """Sec. 3.2 'Rasterization' + Eq. depth_affine_camera: key b_z - p_z ascending."""
    rng = np.random.default_rng(1)
    z = rng.uniform(-5, 80, size=500).astype(np.float32)
    z[100:140] = z[5]          # ties
    mean = np.zeros((500, 3), np.float32); mean[:, 2] = z
    order = oracle.depth_order(mean, 90.0)
    kap = (np.float32(90.0) - z).astype(np.float32)
    for a, b in zip(order[:-1], order[1:]):
        assert kap[a] < kap[b] or (kap[a] == kap[b] and a < b)
    assert sorted(order.tolist()) == list(range(500))


# ---------------------------------------------------------------- P5 depth
def test_p5_depth_is_line_plane_intersection_altitude():
    """Eqs. affine2dgs_uv2screen + depth_affine_camera: D / w is b_z minus the altitude
    where the affine pixel ray {p : B_xy p + b_xy = x} meets the surfel plane."""
    W, H = 32, 32
    F = np.array([[1.6, 0.5, -0.6, 16.0], [0.3, -1.8, 0.7, 15.0]], np.float32)
    n = np.array([0.4, 0.2, 1.0]); n /= np.linalg.norm(n)
    tu = np.cross(n, [0.0, 1.0, 0.0]); tu /= np.linalg.norm(tu)
    tv = np.cross(n, tu)
    p = np.array([0.3, 0.2, 6.0])
    sc = custom_scene([dict(p=p, tu=tu, tv=tv, s=(4.0, 3.0), o=0.6, a=(1, 1, 1))], [(W, H, F)],
                      bz=40.0)
    out = oracle.forward(sc, Settings(lowpass_mode=1))
    w = planar(out, "albedo", W, H, 3)[0]
    D = planar(out, "depth", W, H, 1)
    B, b = F[:, :3].astype(np.float64), F[:, 3].astype(np.float64)
    pk = np.float32(p).astype(np.float64)
    nk = np.cross(np.float32(tu).astype(np.float64), np.float32(tv).astype(np.float64))
    d = np.cross(B[0], B[1])
    checked = 0
    for j in range(H):
        for i in range(W):
            if w[j, i] < 0.05:
                continue
            p0xy = np.linalg.solve(B[:, :2], np.array([i + 0.5, j + 0.5]) - b)
            p0 = np.array([p0xy[0], p0xy[1], 0.0])
            t = nk @ (pk - p0) / (nk @ d)
            z_int = (p0 + t * d)[2]
            assert abs(D[j, i] / w[j, i] - (np.float32(40.0) - z_int)) < 1e-9
            checked += 1
    assert checked > 30


# ---------------------------------------------------------------- P6 sun camera
def test_p6_sun_direction_is_nullspace_of_sun_camera():
    """Supp. A: s = (cos phi / tan theta, sin phi / tan theta, 1) satisfies B_sun s = 0 and
    B_sun p = lam * B_xy p' with p' = p - p_z s on the z = 0 plane."""
    sc = synth.make_scene(synth.tiny(n_surfels=200, views=((30, 30), (41, 23))))
    for v in range(2):
        Bs, bs, zfar = oracle.sun_camera(sc, v, S=512)
        phi, th = sc["sun"][v].astype(np.float64)
        s = np.array([math.cos(phi) / math.tan(th), math.sin(phi) / math.tan(th), 1.0])
        assert np.abs(Bs @ s).max() < 1e-12 * np.abs(Bs).max()
        B, b = oracle.view_camera(sc, v)
        lam = Bs[0, 0] / B[0, 0]
        rng = np.random.default_rng(v)
        for _ in range(5):
            P = rng.normal(size=3) * 10
            pf = P - P[2] * s
            assert abs(pf[2]) < 1e-15
            np.testing.assert_allclose(Bs @ P, lam * (B @ pf), rtol=1e-12, atol=1e-9)
        mean = sc["surfels"]["mean"].astype(np.float64)
        xs = mean @ Bs.T + bs
        assert xs.min() >= 0 and xs.max() < 512
        assert zfar == pytest.approx(sc["b_z"] - mean[:, 2].min() + 10.0)


# ---------------------------------------------------------------- P7 box shadow
def _box_scene(h, phi, theta, spacing=0.8, half=14.0, box=(-3.0, 3.0, -3.0, 3.0)):
    surf = []
    xs = np.arange(-half, half + 1e-9, spacing)
    x0, x1, y0, y1 = box
    for x in xs:
        for y in xs:
            if x0 <= x <= x1 and y0 <= y <= y1:
                continue
            surf.append(dict(p=(x, y, 0.0), tu=(1, 0, 0), tv=(0, 1, 0), s=(0.6, 0.6), o=0.95, a=(.5, .5, .5)))
    bx = np.arange(x0, x1 + 1e-9, spacing / 2)
    by = np.arange(y0, y1 + 1e-9, spacing / 2)
    for x in bx:
        for y in by:
            surf.append(dict(p=(x, y, h), tu=(1, 0, 0), tv=(0, 1, 0), s=(0.4, 0.4), o=0.95, a=(.8, .8, .8)))
    for zz in np.arange(spacing / 2, h, spacing / 2):
        for x in bx:
            for y, nrm in ((y0, -1), (y1, 1)):
                surf.append(dict(p=(x, y, zz), tu=(1, 0, 0), tv=(0, 0, 1), s=(0.4, 0.4), o=0.95, a=(.5, .5, .5)))
        for y in by:
            for x in (x0, x1):
                surf.append(dict(p=(x, y, zz), tu=(0, 1, 0), tv=(0, 0, 1), s=(0.4, 0.4), o=0.95, a=(.5, .5, .5)))
    F = nadir(0.25, 128, 128)
    return custom_scene(surf, [(128, 128, F)], bz=h + 10.0,
                        sun=np.array([[phi, theta]], np.float32))


def _in_shadow(q, h, phi, theta, box):
    """Closed form: the ground point q is shadowed iff the segment from q towards the sun,
    up to altitude h, crosses the box footprint (shadow length h / tan(theta))."""
    x0, x1, y0, y1 = box
    L = h / math.tan(theta)
    ts = np.linspace(0.0, 1.0, 400)
    px = q[0] + ts * L * math.cos(phi)
    py = q[1] + ts * L * math.sin(phi)
    return bool(np.any((px >= x0) & (px <= x1) & (py >= y0) & (py <= y1)))


def _dist_to_boundary(q, h, phi, theta, box):
    best = np.inf
    for dx in np.linspace(-1, 1, 9):
        for dy in np.linspace(-1, 1, 9):
            r = math.hypot(dx, dy)
            if r == 0:
                continue
            if _in_shadow((q[0] + dx * 2.5 / r, q[1] + dy * 2.5 / r), h, phi, theta, box) != \
               _in_shadow(q, h, phi, theta, box):
                best = min(best, 2.5)
    return best


@pytest.mark.parametrize("phi_deg,theta_deg", [(30.0, 45.0), (200.0, 35.0)])
def test_p7_box_shadow_matches_closed_form_away_from_edges(phi_deg, theta_deg):
    h, box = 8.0, (-3.0, 3.0, -3.0, 3.0)
    phi, theta = math.radians(phi_deg), math.radians(theta_deg)
    sc = _box_scene(h, phi, theta, box=box)
    mean = sc["surfels"]["mean"]
    sel = np.where((mean[:, 2] == 0.0) & (np.abs(mean[:, 0]) < 11) & (np.abs(mean[:, 1]) < 11))[0]
    vis = oracle.shadow(sc, 0, Settings(sun_map_size=256), sel=sel)
    agree = total = n_shadow = 0
    for k, v in zip(sel, vis):
        q = mean[k, :2].astype(np.float64)
        if _dist_to_boundary(q, h, phi, theta, box) < np.inf:
            continue              # within 2.5 m (about two surfel supports) of the edge
        expect = not _in_shadow(q, h, phi, theta, box)
        total += 1
        n_shadow += not expect
        agree += (v >= 0.5) == expect
    assert total > 200 and n_shadow > 15
    assert agree == total
    # P14: roof of the (only, tallest) box is lit
    roof = np.where(mean[:, 2] == np.float32(h))[0][:40]
    assert np.all(oracle.shadow(sc, 0, Settings(sun_map_size=256), sel=roof) >= 0.5)


# ---------------------------------------------------------------- P8 finite differences
def _loss(sc, dI, dD, dN, vis, st):
    out = oracle.forward(sc, st, vis=vis)
    order = oracle.depth_order(sc["surfels"]["mean"], sc["b_z"])
    key = np.concatenate([out["count"], order])
    return (out["image"] @ dI + out["depth"] @ dD + out["normal"] @ dN), key


def test_p8_adjoint_matches_central_differences():
    """The analytic adjoint (reverse sweep of Eq. rasterization + chain rule through
    Eqs. affine2dgs_Qq, depth_affine_camera, image_formation and F' = F + dF) equals
    FP64 central differences of the forward."""
    sc = synth.make_scene(synth.tiny(n_surfels=120, views=((26, 22), (19, 24)), seed=11))
    V = 2
    rng = np.random.default_rng(5)
    vis = rng.uniform(0.0, 1.0, size=(V, 120)).astype(np.float32)
    dI, dD, dN = [x.astype(np.float64) for x in synth.upstream_grads(sc)]
    st = ST
    g = oracle.backward(sc, dI, dD, dN, st, vis=vis)
    base_out = oracle.forward(sc, st, vis=vis)
    assert not base_out["ambiguous"].any()
    groups = [("mean", sc["surfels"], "mean"), ("t_u", sc["surfels"], "t_u"),
              ("t_v", sc["surfels"], "t_v"), ("scale", sc["surfels"], "scale"),
              ("opacity", sc["surfels"], "opacity"), ("albedo", sc["surfels"], "albedo"),
              ("dF", sc, "dF"), ("colC", sc, "colC"), ("colc", sc, "colc"), ("ambient", sc, "ambient")]
    checked = 0
    for name, holder, key in groups:
        arr = holder[key]
        flat = arr.reshape(-1)
        gg = g[name].reshape(-1)
        rms = np.sqrt(np.mean(gg ** 2)) + 1e-30
        idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            x0 = flat[i]
            h = np.float32(max(1.0, abs(float(x0))) * 1e-5)
            xp, xm = np.float32(x0 + h), np.float32(x0 - h)
            flat[i] = xp
            lp, cp = _loss(sc, dI, dD, dN, vis, st)
            flat[i] = xm
            lm, cm = _loss(sc, dI, dD, dN, vis, st)
            flat[i] = x0
            if not np.array_equal(cp, cm):
                continue          # a discrete decision (skip, stop, order) flipped
            fd = (lp - lm) / (np.float64(xp) - np.float64(xm))
            err = abs(fd - gg[i]) / max(abs(gg[i]), 1e-2 * rms)
            assert err < 1e-5, (name, i, fd, gg[i])
            checked += 1
    assert checked > 90


# ---------------------------------------------------------------- P9 colour identity
def test_p9_identity_colour_and_full_visibility_give_albedo():
    """Eq. image_formation with C = I, c = 0 (initialisation) and V = 1: I = A."""
    sc = synth.make_scene(synth.tiny(n_surfels=200, views=((21, 19),)))
    sc["colC"] = np.eye(3, dtype=np.float32)[None].copy()
    sc["colc"] = np.zeros((1, 3), np.float32)
    out = oracle.forward(sc, ST)
    np.testing.assert_array_equal(out["image"], out["albedo"])


def test_image_formation_with_shadow_and_ambient():
    """Eq. image_formation: (C A + c) * (V + (1 - V) L_a), per pixel and channel."""
    sc = synth.make_scene(synth.tiny(n_surfels=200, views=((21, 19),)))
    vis = np.random.default_rng(2).uniform(size=(1, 200)).astype(np.float32)
    out = oracle.forward(sc, ST, vis=vis)
    P = 21 * 19
    A = out["albedo"].reshape(3, P)
    V = out["vis"]
    C = sc["colC"][0].astype(np.float64); c = sc["colc"][0].astype(np.float64)
    La = sc["ambient"][0].astype(np.float64)
    expect = (C @ A + c[:, None]) * (V[None] + (1 - V[None]) * La[:, None])
    np.testing.assert_allclose(out["image"].reshape(3, P), expect, atol=1e-13)


# ---------------------------------------------------------------- P10 culling
def test_p10_transparent_surfels_have_no_tiles_and_no_effect_and_empty_scene():
    sc = synth.make_scene(synth.tiny(n_surfels=150, views=((24, 24),)))
    base = oracle.forward(sc, ST)
    s2 = {k: np.concatenate([v, v[:20]]) for k, v in sc["surfels"].items()}
    s2["opacity"][150:] = np.float32(1.0 / 255.0) * np.float32(0.99)
    sc2 = dict(sc, surfels=s2)
    out = oracle.forward(sc2, ST)
    np.testing.assert_allclose(out["image"], base["image"], atol=1e-15)
    B, b = oracle.view_camera(sc2, 0)
    _, _, pix, tiles = oracle.binning(sc2, B, b, 24, 24, 16, ST)
    assert np.all(tiles[150:, 0] > tiles[150:, 1])
    empty = dict(sc, surfels={k: v[:0] for k, v in sc["surfels"].items()})
    e = oracle.forward(empty, ST)
    assert np.all(e["T"] == 1.0) and np.all(e["albedo"] == 0.0)


# ---------------------------------------------------------------- P11 camera delta
def test_p11_delta_translation_shifts_the_image():
    """Sec. 3.3: the last column of dF_xy translates the image: rendering with
    b + (dx, dy) equals the original render sampled at x - (dx, dy)."""
    sc = synth.make_scene(synth.tiny(n_surfels=250, views=((30, 26),)))
    sc["dF"][:] = 0
    base = oracle.forward(sc, ST)
    sc2 = dict(sc, dF=sc["dF"].copy())
    sc2["dF"][0, 0, 3] = 3.0
    sc2["dF"][0, 1, 3] = -2.0
    out = oracle.forward(sc2, ST)
    W, H = 30, 26
    a = base["image"].reshape(3, H, W)
    b = out["image"].reshape(3, H, W)
    np.testing.assert_allclose(b[:, 0:H - 2, 3:W], a[:, 2:H, 0:W - 3], atol=1e-12)


# ---------------------------------------------------------------- P13 binning box
def test_p13_binning_box_contains_every_contributing_pixel():
    """Sec. 3.2 'Rasterization' (screen-space bounding box per splat): brute force over
    single-surfel renders; every pixel a surfel reaches lies in its FP64 box."""
    sc = synth.make_scene(synth.tiny(n_surfels=60, views=((48, 44),), seed=3))
    s = sc["surfels"]
    s["t_v"][:6] = np.array([0, 0, 1], np.float32)         # some edge-on / near-degenerate
    s["t_u"][:6] = np.array([1, 0, 0], np.float32)
    B, b = oracle.view_camera(sc, 0)
    for mode in (0, 1):
        st = Settings(lowpass_mode=mode)
        _, _, pix, _ = oracle.binning(sc, B, b, 48, 44, 16, st)
        for k in range(60):
            one = dict(sc, surfels={kk: v[k:k + 1] for kk, v in s.items()},
                       colC=None, colc=None, ambient=None)
            out = oracle.forward(one, st)
            hit = out["count"].reshape(44, 48) > 0
            jj, ii = np.nonzero(hit)
            if ii.size == 0:
                continue
            assert pix[k, 0] <= ii.min() and ii.max() <= pix[k, 1]
            assert pix[k, 2] <= jj.min() and jj.max() <= pix[k, 3]


def test_p13_binning_box_is_tight():
    """Sec. 3.2 'Rasterization': the FP64 box is no wider than the support it bounds.
    The support is sampled on a quarter-pixel lattice by rendering each surfel alone with
    the camera translated by multiples of 1/4 px (the camera-delta translation column,
    Sec. 3.3: b - d renders the image at x + d); the box may extend past the sampled
    support by at most 1 px (pixel rounding) plus the lattice step on each side."""
    W, H, q = 48, 44, 4
    sc = synth.make_scene(synth.tiny(n_surfels=40, views=((W, H),), seed=3))
    s = sc["surfels"]
    s["t_v"][:4] = np.array([0, 0, 1], np.float32)         # edge-on: low-pass disk only
    s["t_u"][:4] = np.array([1, 0, 0], np.float32)
    B, b = oracle.view_camera(sc, 0)
    checked = 0
    for mode in (0, 1):
        st = Settings(lowpass_mode=mode)
        _, _, pix, _ = oracle.binning(sc, B, b, W, H, 16, st)
        for k in range(40):
            one = dict(sc, surfels={kk: v[k:k + 1] for kk, v in s.items()},
                       colC=None, colc=None, ambient=None)
            xs, ys = [], []
            for a in range(q):
                for c in range(q):
                    one["dF"] = sc["dF"].copy()
                    one["dF"][0, 0, 3] -= np.float32(a / q)
                    one["dF"][0, 1, 3] -= np.float32(c / q)
                    hit = oracle.forward(one, st)["count"].reshape(H, W) > 0
                    jj, ii = np.nonzero(hit)
                    xs.extend(ii + 0.5 + a / q)
                    ys.extend(jj + 0.5 + c / q)
            if pix[k, 0] > pix[k, 1]:
                continue
            assert xs, f"surfel {k}: non-empty box but no support sample"
            slack = 1.0 + 1.0 / q
            assert pix[k, 0] + 0.5 >= min(xs) - slack and pix[k, 1] + 0.5 <= max(xs) + slack, k
            assert pix[k, 2] + 0.5 >= min(ys) - slack and pix[k, 3] + 0.5 <= max(ys) + slack, k
            checked += 1
    assert checked > 40


def test_tile_lists_from_ranges_small_example():
    order = np.array([2, 0, 1])
    tiles = np.array([[0, 1, 0, 0], [1, 1, 0, 1], [0, 0, 0, 1]], np.int32)
    rng, flat = oracle.tile_lists(order, tiles, 20, 20, 16)    # 2x2 tiles
    lists = [flat[s:e].tolist() for s, e in rng]
    assert lists == [[2, 0], [0, 1], [2], [1]]
