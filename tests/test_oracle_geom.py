"""Pins of the oracle's geometric regularisers: the depth distortion (the loss term the
paper weights with 0.05 in Supp. B, in the squared 2DGS form) and the depth-gradient
normal with its normal-consistency loss (Sec. 3.2 "Normal Definition", Eq.
surface_normal).

* closed forms: two stacked discs under a nadir camera give w1 w2 (m1 - m2)^2 at every
  pixel; one disc gives no distortion; the depth normal of a planar surfel is the
  plane's normal and its loss is the mean final transmittance over valid pixels;
* an independent second statement of both definitions (dense torch FP64: the moment
  form of the distortion, a linear solve for the back-projection) with autograd;
* FP64 central differences of the whole chain (render -> distortion / depth normals ->
  loss) on entries whose step crosses no discrete decision.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import Settings, dense, geom
from test_oracle_pins import F32, custom_scene, nadir, pixel_centres


def _alpha_nadir(o, su, sv, g, cx, cy, xs, ys):
    """P1 closed form: axis-aligned Gaussian of a horizontal disc under a nadir camera."""
    dx = (xs - cx) * g
    dy = (ys - cy) * g
    return np.minimum(F32(0.99), F32(o) * np.exp(-0.5 * ((dx / F32(su)) ** 2 + (dy / F32(sv)) ** 2)))


def test_distortion_of_two_stacked_discs_is_closed_form():
    g, W, H, ds = 0.5, 30, 26, 0.05
    bz = 50.0
    up = dict(p=(0.4, -0.3, 9.0), tu=(1, 0, 0), tv=(0, 1, 0), s=(3.0, 2.5), o=0.7, a=(1, 0, 0))
    lo = dict(p=(0.4, -0.3, 2.0), tu=(1, 0, 0), tv=(0, 1, 0), s=(2.6, 3.1), o=0.8, a=(0, 1, 0))
    F = nadir(g, W, H)
    st = Settings(depth_scale=ds)
    sc = custom_scene([lo, up], [(W, H, F)], bz=bz)
    out = oracle.forward(sc, st, with_dist=True)
    xs, ys = pixel_centres(W, H)
    # pixel coordinates of the common centre under the nadir camera x = p/g + W/2, -p/g + H/2
    cx = F32(0.4) / F32(g) + W / 2
    cy = -F32(-0.3) / F32(g) + H / 2
    a1 = _alpha_nadir(0.7, 3.0, 2.5, F32(g), cx, cy, xs, ys)     # upper disc, first
    a2 = _alpha_nadir(0.8, 2.6, 3.1, F32(g), cx, cy, xs, ys)
    amin = Settings().alpha_min
    both = (a1 >= amin) & (a2 >= amin)
    m1 = (F32(bz) - F32(9.0)) * ds
    m2 = (F32(bz) - F32(2.0)) * ds
    expect = np.where(both, a1 * a2 * (1 - a1) * (m1 - m2) ** 2, 0.0)
    ok = ~out["ambiguous"]
    assert both.sum() > 200
    np.testing.assert_allclose(out["dist"][ok], expect.reshape(-1)[ok], rtol=1e-12, atol=1e-15)
    one = oracle.forward(custom_scene([up], [(W, H, F)], bz=bz), st, with_dist=True)
    assert np.all(one["dist"] == 0.0)


def _tiny(seed=5, n=90, views=((21, 17), (16, 19))):
    return synth.make_scene(synth.tiny(n_surfels=n, views=views, seed=seed))


def test_distortion_c_oracle_matches_dense_moment_form_and_autograd():
    sc = _tiny()
    st = Settings(depth_scale=0.07)
    out = oracle.forward(sc, st, with_dist=True)
    P = dense.params_from_scene(sc)
    r = dense.render(P, sc, st)
    dist = torch.cat([x["dist"].reshape(-1) for x in r])
    ok = ~out["ambiguous"]
    assert out["dist"].max() > 1e-3
    np.testing.assert_allclose(dist.detach().numpy()[ok], out["dist"][ok], atol=1e-12)
    gd = np.random.default_rng(3).standard_normal(out["dist"].shape[0]).astype(np.float32)
    z = np.zeros_like(out["depth"])
    g = oracle.backward(sc, np.zeros(3 * z.size), z, np.zeros(3 * z.size), st, dDist=gd)
    (dist * torch.as_tensor(gd.astype(np.float64))).sum().backward()
    for k in ("mean", "t_u", "t_v", "scale", "opacity", "dF"):
        a = P[k].grad.numpy().reshape(-1)
        b = g[k].reshape(-1)
        assert np.abs(a - b).max() <= 1e-10 * max(np.abs(a).max(), 1e-30), k
    assert np.abs(g["albedo"]).max() == 0.0      # the distortion does not see colour


def _fd_check(sc, loss_fn, g, rng, per_group=10, tol=1e-5):
    groups = [("mean", sc["surfels"]), ("t_u", sc["surfels"]), ("t_v", sc["surfels"]),
              ("scale", sc["surfels"]), ("opacity", sc["surfels"]), ("dF", sc)]
    _, k0 = loss_fn(sc)
    checked = 0
    for name, holder in groups:
        flat = holder[name].reshape(-1)
        gg = g[name].reshape(-1)
        rms = np.sqrt(np.mean(gg ** 2)) + 1e-30
        for i in rng.choice(flat.size, size=min(per_group, flat.size), replace=False):
            x0 = flat[i]
            # camera entries are ~1e-2 px/m: a step of 1e-5 is a 0.1 % change of the
            # projection, where the truncation error of the difference shows
            h = np.float32(1e-6 if name == "dF" else max(1.0, abs(float(x0))) * 1e-5)
            xp, xm = np.float32(x0 + h), np.float32(x0 - h)
            flat[i] = xp
            lp, kp = loss_fn(sc)
            flat[i] = xm
            lm, km = loss_fn(sc)
            flat[i] = x0
            if not (np.array_equal(kp, k0) and np.array_equal(km, k0)):
                continue
            fd = (lp - lm) / (np.float64(xp) - np.float64(xm))
            err = abs(fd - gg[i]) / max(abs(gg[i]), 1e-2 * rms)
            assert err < tol, (name, i, fd, gg[i])
            checked += 1
    return checked


def test_distortion_adjoint_matches_central_differences():
    sc = _tiny(seed=9)
    st = Settings(depth_scale=0.07)
    base = oracle.forward(sc, st, with_dist=True)
    gd = np.random.default_rng(4).standard_normal(base["dist"].shape[0]).astype(np.float32)
    z = np.zeros_like(base["depth"])
    g = oracle.backward(sc, np.zeros(3 * z.size), z, np.zeros(3 * z.size), st, dDist=gd)

    def loss(s):
        o = oracle.forward(s, st, with_dist=True)
        order = oracle.depth_order(s["surfels"]["mean"], s["b_z"])
        return o["dist"] @ gd.astype(np.float64), np.concatenate([o["sig"].view(np.int64), order])

    assert _fd_check(sc, loss, g, np.random.default_rng(6)) > 40


def test_depth_normal_of_a_planar_surfel_is_its_normal():
    """A large tilted disc seen by an oblique affine camera: on its uv branch the depth is
    affine in the pixel position (Eq. depth_affine_camera on Eq. affine2dgs_uv2screen), so
    the back-projected points lie on the disc's plane and Eq. surface_normal returns the
    plane normal; with N_r = w n and w = 1 - T the loss is the mean of T over valid
    pixels."""
    W, H = 40, 34
    tu = np.array([0.96, 0.0, 0.28]); tu /= np.linalg.norm(tu)
    tv = np.array([0.1, 0.97, -0.2]); tv -= tu * (tv @ tu); tv /= np.linalg.norm(tv)
    disc = dict(p=(0.0, 0.0, 3.0), tu=tuple(tu), tv=tuple(tv), s=(40.0, 40.0), o=0.98, a=(1, 1, 1))
    # oblique camera: view direction 20 deg off nadir, image axes orthogonal to it
    nu = np.deg2rad(20.0)
    e1 = np.array([np.cos(nu), 0.0, np.sin(nu)])
    e2 = np.array([0.0, -1.0, 0.0])
    g = 1.5
    F = [list(e1 / g) + [W / 2], list(e2 / g) + [H / 2]]
    sc = custom_scene([disc], [(W, H, F)], bz=60.0)
    out = oracle.forward(sc, Settings())
    loss, Nd, gD, gN, gF = geom.normal_loss(sc, out["depth"], out["T"], out["normal"], tau=0.5)
    Nd = Nd.reshape(3, H, W)
    n = np.cross(F32(disc["tu"]), F32(disc["tv"]))
    n /= np.linalg.norm(n)
    d = np.cross(F32(F[0][:3]), F32(F[1][:3]))
    d = -d if d[2] > 0 else d
    n = -n if n @ d > 0 else n
    T = out["T"].reshape(H, W)
    cover = (1 - T) >= 0.5
    valid = np.zeros((H, W), bool)
    valid[1:-1, 1:-1] = cover[1:-1, 1:-1] & cover[1:-1, 2:] & cover[1:-1, :-2] & cover[2:, 1:-1] & cover[:-2, 1:-1]
    assert valid.sum() > 0.8 * (W - 2) * (H - 2)
    np.testing.assert_allclose(Nd[:, valid].T, np.broadcast_to(n, (valid.sum(), 3)), atol=1e-9)
    np.testing.assert_allclose(loss[0], T[valid].sum() / (W * H), rtol=1e-9)


def test_normal_loss_adjoint_matches_dense_autograd():
    sc = _tiny(seed=13, n=160, views=((23, 19), (18, 21)))
    out = oracle.forward(sc, Settings())
    loss, Nd, gD, gN, gF = geom.normal_loss(sc, out["depth"], out["T"], out["normal"], tau=0.3)
    W, H = sc["width"], sc["height"]
    off = 0
    total = 0.0
    for v in range(len(W)):
        w, h = int(W[v]), int(H[v])
        P = w * h
        D = torch.tensor(out["depth"][off:off + P].reshape(h, w), requires_grad=True)
        T = torch.tensor(out["T"][off:off + P].reshape(h, w))
        N = torch.tensor(out["normal"][3 * off:3 * off + 3 * P].reshape(3, h, w), requires_grad=True)
        dF = torch.tensor(sc["dF"][v].astype(np.float64), requires_grad=True)
        L = dense.normal_loss(D, T, N, sc["Fxy"][v], dF, float(sc["b_z"]), tau=0.3)
        L.backward()
        assert abs(L.item() - loss[v]) <= 1e-12
        np.testing.assert_allclose(gD[off:off + P], D.grad.numpy().reshape(-1), atol=1e-12)
        np.testing.assert_allclose(gN[3 * off:3 * off + 3 * P], N.grad.numpy().reshape(-1), atol=1e-12)
        np.testing.assert_allclose(gF[v], dF.grad.numpy(), rtol=1e-9, atol=1e-12)
        total += L.item()
        off += P
    assert total > 0.01 and np.abs(gF).max() > 0


def test_normal_loss_end_to_end_central_differences():
    """d/dtheta of sum_v L_v(render(theta)) with the accumulated opacity held at its value
    (the stop-gradient reading): the loss's map adjoints pulled back through the render's
    adjoint, plus the camera term, against FP64 central differences."""
    sc = _tiny(seed=21, n=160, views=((22, 20), (19, 18)))
    st = Settings()
    base = oracle.forward(sc, st)
    tau = 0.3
    T0 = base["T"].copy()
    _, _, gD, gN, gF = geom.normal_loss(sc, base["depth"], T0, base["normal"], tau=tau)
    P = gD.size
    g = oracle.backward(sc, np.zeros(3 * P), gD, gN, st)
    g["dF"] = g["dF"] + gF

    def loss(s):
        o = oracle.forward(s, st)
        L = geom.normal_loss(s, o["depth"], T0, o["normal"], tau=tau)[0].sum()
        order = oracle.depth_order(s["surfels"]["mean"], s["b_z"])
        return L, np.concatenate([o["sig"].view(np.int64), order])

    assert _fd_check(sc, loss, g, np.random.default_rng(8), per_group=12) > 45
