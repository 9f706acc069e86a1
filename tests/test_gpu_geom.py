"""GPU parity of the geometric regularisers (HIP kernels through the C ABI) against the
FP64 oracle: the depth distortion composited by the raster forward and its adjoint in the
raster backward, and the depth-gradient normals with the normal-consistency loss (Sec.
3.2 "Normal Definition", Eq. surface_normal) computed on the rendered maps.

Bars: maps (distortion, depth normals) max-abs 1e-4 on non-ambiguous pixels; losses rel
1e-5; gradients per tensor rel 1e-3 (the metric of the raster tests)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import geom
from gpu_common import GRAD_KEYS, expand3, make_plan, oracle_settings, rel_err, to_np

pytestmark = pytest.mark.gpu


def scene(seed=5, n=400, views=((45, 38), (33, 29), (40, 41))):
    return synth.make_scene(synth.tiny(n_surfels=n, views=views, seed=seed))


def depth_scale(sc):
    return float(np.float32(2.0 / sc["spec"].extent))


def cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device="cuda")


@pytest.mark.parametrize("ts,batch", [(8, 64), (16, 64), (8, 48), (32, 100)])
def test_distortion_forward_and_backward_match_oracle(ts, batch):
    sc = scene()
    ds = depth_scale(sc)
    n, V = sc["surfels"]["mean"].shape[0], len(sc["width"])
    vis = np.random.default_rng(2).uniform(size=(V, n)).astype(np.float32)
    plan, surf, views = make_plan(sc, ts=ts, batch=batch)
    st = oracle_settings(ts=ts)
    st.depth_scale = ds
    plain = plan.forward(surf, views, cuda(vis))
    plain = {k: to_np(t) for k, t in plain.items()}
    out = plan.forward(surf, views, cuda(vis), depth_scale=ds)
    ref = oracle.forward(sc, st, vis=vis, with_dist=True)
    ok = ~ref["ambiguous"]
    o = {k: to_np(t) for k, t in out.items()}
    # the channel changes nothing else
    for k in ("image", "albedo", "vis", "depth", "normal", "T", "last"):
        assert np.array_equal(o[k], plain[k]), k
    assert ref["dist"].max() > 1e-3
    np.testing.assert_allclose(o["dist"][ok], ref["dist"][ok], atol=1e-4)
    # backward with image, depth, normal and distortion upstream gradients
    dI, dD, dN = synth.upstream_grads(sc)
    okI = expand3(ok, sc["width"], sc["height"])
    dI, dD, dN = dI * okI, dD * ok, dN * okI
    gd = (np.random.default_rng(7).standard_normal(ok.size) * ok).astype(np.float32)
    g = plan.backward(surf, views, out, cuda(dI), cuda(dD), cuda(dN), vis=cuda(vis),
                      depth_scale=ds, d_dist=cuda(gd))
    gr = oracle.backward(sc, dI, dD, dN, st, vis=vis, dDist=gd)
    for k in GRAD_KEYS:
        assert rel_err(to_np(g[k]), gr[k]) < 1e-3, k
    # the distortion's own share: distortion gradient alone
    z = torch.zeros_like(out["depth"])
    g2 = plan.backward(surf, views, out, torch.zeros_like(out["image"]), z,
                       torch.zeros_like(out["normal"]), vis=cuda(vis), depth_scale=ds,
                       d_dist=cuda(gd))
    z0 = np.zeros_like(dD)
    gr2 = oracle.backward(sc, np.zeros_like(dI), z0, np.zeros_like(dN), st, vis=vis, dDist=gd)
    for k in ("mean", "t_u", "t_v", "scale", "opacity", "dF"):
        assert np.abs(gr2[k]).max() > 0, k
        assert rel_err(to_np(g2[k]), gr2[k]) < 1e-3, k


# the kernel walks blocks of 256 columns x 16 rows: the larger views span two blocks
# across (ragged second, halo columns at the seam) and end in ragged row bands; views of
# 1 x 5 and 3 x 3 pixels have no interior pixel or one
@pytest.mark.parametrize("n,views", [(400, ((45, 38), (33, 29), (40, 41))),
                                     (3000, ((300, 290), (270, 263))),
                                     (400, ((1, 5), (3, 3), (40, 41)))])
def test_normal_loss_kernel_matches_oracle_on_the_same_maps(n, views):
    sc = scene(seed=11, n=n, views=views)
    plan, surf, views = make_plan(sc, ts=8)
    out = plan.forward(surf, views)
    maps = {k: to_np(out[k]).astype(np.float64) for k in ("depth", "T", "normal")}
    P, V = views.pixels, len(sc["width"])
    rng = np.random.default_rng(3)
    base_d = rng.standard_normal(P).astype(np.float32)
    base_n = rng.standard_normal(3 * P).astype(np.float32)
    base_f = rng.standard_normal((V, 2, 4)).astype(np.float32)
    w, tau = 0.7, 0.4
    loss, gD, gN, gF, Nd = plan.normal_loss(views, out, weight=w, tau=tau, normal_d=True)
    rl, rNd, rgD, rgN, rgF = geom.normal_loss(sc, maps["depth"], maps["T"], maps["normal"], tau=tau)
    valid = np.abs(rNd).reshape(-1) > 0
    assert valid.mean() > 0.3
    np.testing.assert_allclose(to_np(loss), w * rl, rtol=1e-5)
    np.testing.assert_allclose(to_np(Nd), rNd, atol=1e-5)
    assert rel_err(to_np(gD), w * rgD) < 1e-4
    assert rel_err(to_np(gN), w * rgN) < 1e-4
    assert rel_err(to_np(gF), w * rgF) < 1e-3
    # gradients are added to the buffers' contents: one FP32 addition per element
    _, gD2, gN2, gF2, _ = plan.normal_loss(views, out, weight=w, tau=tau, d_depth=cuda(base_d),
                                           d_normal=cuda(base_n), d_dF=cuda(base_f))
    assert np.array_equal(to_np(gD2), base_d + to_np(gD))
    assert np.array_equal(to_np(gN2), base_n + to_np(gN))
    assert np.array_equal(to_np(gF2), base_f + to_np(gF))


def test_geometric_losses_end_to_end_gradients_match_oracle():
    """Forward with distortion -> normal-consistency loss on the maps -> backward with the
    distortion's and the loss's upstream gradients, all on the GPU, against the same
    chain in the oracle."""
    sc = scene(seed=24, n=500, views=((36, 31), (30, 34)))
    ds = depth_scale(sc)
    st = oracle_settings(ts=8)
    st.depth_scale = ds
    ref = oracle.forward(sc, st, with_dist=True)
    assert not ref["ambiguous"].any()
    plan, surf, views = make_plan(sc, ts=8)
    out = plan.forward(surf, views, depth_scale=ds)
    w_n, w_d, tau = 0.05, 0.05, 0.5
    P = views.pixels
    gd = torch.full((P,), w_d, dtype=torch.float32, device="cuda")
    loss, dD, dN, dF_n, _ = plan.normal_loss(views, out, weight=w_n, tau=tau)
    g = plan.backward(surf, views, out, torch.zeros_like(out["image"]), dD, dN,
                      depth_scale=ds, d_dist=gd)
    rl, _, rgD, rgN, rgF = geom.normal_loss(sc, ref["depth"], ref["T"], ref["normal"], tau=tau)
    np.testing.assert_allclose(to_np(loss), w_n * rl, rtol=1e-4)
    np.testing.assert_allclose(float(to_np(out["dist"]).sum()) * w_d, float(ref["dist"].sum()) * w_d,
                               rtol=1e-4)
    gr = oracle.backward(sc, np.zeros(3 * P), w_n * rgD, w_n * rgN, st,
                         dDist=np.full(P, w_d, np.float32))
    gr["dF"] = gr["dF"] + w_n * rgF
    gg = {k: to_np(g[k]) for k in GRAD_KEYS}
    gg["dF"] = gg["dF"] + to_np(dF_n)
    for k in ("mean", "t_u", "t_v", "scale", "opacity", "dF"):
        assert np.abs(gr[k]).max() > 0, k
        assert rel_err(gg[k], gr[k]) < 1e-3, k
