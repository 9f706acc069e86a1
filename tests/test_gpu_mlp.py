"""GPU parity of the surrogate MLP (MFMA kernels through the C ABI) against the FP64
BF16-emulating oracle, and of the surrogate shadow pass against the geometric pass.

Bars (no tolerance is stated for the learned part; these follow from BF16 rounding):
probabilities within 1e-2 on >= 99.9 % of points; weight gradients per tensor with
relative L2 error <= 1e-2; Adam to FP32 rounding."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp as om
import paper_2606_28581_amd as ss
from paper_2606_28581_amd import surrogate as sg
from gpu_common import context, make_plan, to_np

pytestmark = pytest.mark.gpu

CENTRE = np.array([3.0, -1.0, 12.0], np.float32)
INV_HALF = np.float32(1.0 / 80.0)


def pts_suns(M, seed):
    rng = np.random.default_rng(seed)
    pts = (rng.uniform(-80, 80, size=(M, 3)) + CENTRE).astype(np.float32)
    sun = np.stack([rng.uniform(0, 2 * np.pi, M), rng.uniform(0.5, 1.2, M)], 1).astype(np.float32)
    return pts, sun


def cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


@pytest.mark.parametrize("M", [1, 33, 1000])
def test_forward_paired_matches_oracle(M):
    pts, sun = pts_suns(M, M)
    w = om.init_params(5)
    net = sg.Mlp(context(), CENTRE, INV_HALF)
    lg = to_np(net.forward(cuda(w), cuda(pts), cuda(sun)))
    ref, _ = om.forward(w.astype(np.float64), pts, sun, CENTRE, INV_HALF, rounding=True)
    dp = np.abs(sigmoid(lg) - sigmoid(ref))
    assert np.mean(dp <= 1e-2) >= 0.999 and dp.max() < 0.05, dp.max()
    assert np.median(np.abs(lg - ref)) < 5e-3


def test_forward_all_pairs_and_probability_output():
    pts, _ = pts_suns(301, 1)
    _, sun = pts_suns(7, 2)
    w = om.init_params(6)
    net = sg.Mlp(context(), CENTRE, INV_HALF)
    p = to_np(net.forward(cuda(w), cuda(pts), cuda(sun), all_pairs=True, prob=True))
    P = np.tile(pts, (7, 1))
    S = np.repeat(sun, 301, axis=0)
    ref, _ = om.forward(w.astype(np.float64), P, S, CENTRE, INV_HALF, rounding=True)
    dp = np.abs(p - sigmoid(ref))
    assert np.mean(dp <= 1e-2) >= 0.999


@pytest.mark.parametrize("mode", ["bce", "dlogit"])
def test_backward_matches_oracle(mode):
    M = 1500
    pts, sun = pts_suns(M, 11)
    w = om.init_params(7)
    rng = np.random.default_rng(3)
    labels = (rng.uniform(size=M) > 0.5).astype(np.float32)
    dl = rng.normal(size=M).astype(np.float32)
    net = sg.Mlp(context(), CENTRE, INV_HALF, max_points=2048)
    loss = torch.zeros(1, device="cuda")
    if mode == "bce":
        g = to_np(net.backward(cuda(w), cuda(pts), cuda(sun), labels=cuda(labels), scale=1.0 / M,
                               loss=loss))
        ref_loss, gref, _ = om.bce_grad(w.astype(np.float64), pts, sun, labels, CENTRE, INV_HALF)
        assert abs(float(loss.item()) - ref_loss) < 1e-3 * max(1.0, ref_loss)
    else:
        g = to_np(net.backward(cuda(w), cuda(pts), cuda(sun), d_logits=cuda(dl), scale=1.0))
        _, cache = om.forward(w.astype(np.float64), pts, sun, CENTRE, INV_HALF)
        gref = om.backward(cache, dl.astype(np.float64))
    G, R = om.unpack(g), om.unpack(gref)
    for k in om.SIZES:
        rel = np.linalg.norm(G[k] - R[k]) / max(np.linalg.norm(R[k]), 1e-30)
        assert rel <= 1e-2, (k, rel)


def test_adam_matches_oracle():
    rng = np.random.default_rng(0)
    n = 5000
    w = rng.normal(size=n).astype(np.float32)
    m = (rng.normal(size=n) * 0.1).astype(np.float32)
    v = (rng.uniform(size=n) * 0.01).astype(np.float32)
    g = rng.normal(size=n).astype(np.float32)
    tw, tm, tv = cuda(w), cuda(m), cuda(v)
    sg.adam(tw, tm, tv, cuda(g), lr=1e-3, step=3)
    f = lambda x: float(np.float32(x))    # the kernel receives FP32 hyper-parameters
    rw, rm, rv = om.adam(w.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                         g.astype(np.float64), f(1e-3), 3, beta1=f(0.9), beta2=f(0.999), eps=f(1e-8))
    np.testing.assert_allclose(to_np(tm), rm, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(to_np(tv), rv, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(to_np(tw), rw, rtol=1e-5, atol=1e-6)


def test_gpu_training_learns_toy_visibility():
    """The GPU's own forward, backward and Adam fit a separable labelling."""
    M = 4096
    pts, sun = pts_suns(M, 21)
    labels = ((pts[:, 0] - CENTRE[0]) * np.cos(sun[:, 0]) > 0).astype(np.float32)
    net = sg.Mlp(context(), CENTRE, INV_HALF, max_points=M)
    w = cuda(om.init_params(8) * 0.5)
    m, v = torch.zeros_like(w), torch.zeros_like(w)
    P, S, Y = cuda(pts), cuda(sun), cuda(labels)
    for t in range(1, 401):
        g = net.backward(w, P, S, labels=Y, scale=1.0 / M)
        sg.adam(w, m, v, g, lr=3e-3, step=t)
    acc = np.mean((to_np(net.forward(w, P, S)) > 0) == (labels > 0.5))
    assert acc > 0.97, acc


@pytest.mark.parametrize("band", [0.0, 0.1, 0.5])
def test_surrogate_shadow_falls_back_exactly(band):
    sc = synth.make_scene(synth.tiny(n_surfels=600, views=((40, 40), (31, 22)), seed=31))
    S = 64
    plan, surf, views = make_plan(sc, S=S, with_sun=True)
    plain = to_np(plan.shadow(surf, views)).copy()
    half = sc["spec"].extent / 2
    net = sg.Mlp(context(), np.zeros(3, np.float32), np.float32(1.0 / half))
    w = cuda(om.init_params(9) * 0.05)
    vis = to_np(sg.shadow_surrogate(plan, net, w, surf, views, band=band))
    p = to_np(net.forward(w, surf.mean, views.sun, all_pairs=True, prob=True)).reshape(2, -1)
    flagged = np.abs(p - 0.5) < band
    assert flagged.sum() > 0 or band == 0.0      # band 0: only the network runs
    np.testing.assert_array_equal(vis[flagged], plain[flagged])
    np.testing.assert_allclose(vis[~flagged], p[~flagged], rtol=0, atol=0)
    assert plan.stats()["fallback"] == int(flagged.sum())


def test_trained_surrogate_gains_over_the_plain_pass():
    """What the learned part adds.  Trained on the geometric pass's own labels with the
    library's kernels, the network decides most held-out (surfel, sun) pairs on its own,
    so the sun raster runs only for the low-confidence rest; with that fallback its
    lit/shadow decisions agree with the plain pass, and the bare network beats both the
    untrained network and the best constant guess."""
    from paper_2606_28581_amd import surrogate_train as st
    spec = synth.tiny(n_surfels=3000, views=((32, 32),), extent=64.0, n_boxes=6, seed=41,
                      box_height=(4.0, 16.0), box_side=(6.0, 14.0))
    sc = synth.make_scene(spec)
    surf, views = ss.scene_to_device(sc, with_sun=False)
    zc = float(np.mean(sc["surfels"]["mean"][:, 2]))
    net = sg.Mlp(context(), np.array([0.0, 0.0, zc], np.float32), np.float32(2.0 / spec.extent))
    cfg = st.TrainConfig(train_suns=300, points_per_sun=2000, eval_suns=40, batch=8192,
                         epochs=40, lr=1e-2, chunk=20)
    lab = st.ShadowLab(context(), surf, views.Fxy, views.b_z, cfg.chunk, sun_map=256, tile=16)
    quiet = lambda *a, **k: None
    w, tr = st.train(lab, net, cfg, log=quiet)
    ev = st.evaluate(lab, net, w, cfg, log=quiet)
    w0 = torch.as_tensor(st.init_params(cfg.init_seed), device="cuda")
    ev0 = st.evaluate(lab, net, w0, cfg, log=quiet)
    const = max(ev["lit_fraction"], 1.0 - ev["lit_fraction"])
    info = dict(trained=ev, untrained=ev0, best_constant=const, training=tr)
    assert ev["agreement_network_only"] > const + 0.05, info
    assert ev["agreement_network_only"] > ev0["agreement_network_only"] + 0.05, info
    assert ev["fallback_fraction"] < 0.5, info
    assert ev["agreement"] > 0.95, info
