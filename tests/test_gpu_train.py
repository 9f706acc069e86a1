"""GPU parity of the training step (HIP kernels through the C ABI) against the FP64
oracle (oracle/train.py with the render, distortion and normal-loss oracles): surfel
activations and their inverse, the fused activation adjoint + Adam, Adam on the per-view
terms with the camera start step, the L1 image loss, and one whole training step
(Supp. B "Experimental Settings").

Bars: activations and Adam updates to FP32 rounding (rtol 1e-5); losses rel 1e-5;
gradients and the first Adam moments of a whole step per tensor rel 1e-3."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2606_28581_amd as ss
from oracle import geom
from oracle import train as ot
from paper_2606_28581_amd import train as tr
from gpu_common import make_plan, oracle_settings, rel_err, to_np

pytestmark = pytest.mark.gpu


def cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.float32), device="cuda")


def random_raw(n, seed):
    rng = np.random.default_rng(seed)
    raw = rng.standard_normal((n, 13)).astype(np.float32)
    raw[:, 0:3] *= 5.0
    raw[:, 3:5] *= 0.5
    raw[:, 10:13] = rng.uniform(size=(n, 3))
    return raw


def empty_surfels(n):
    f = lambda *s: torch.empty(*s, dtype=torch.float32, device="cuda")
    return ss.SurfelTensors(f(n, 3), f(n, 3), f(n, 3), f(n, 2), f(n), f(n, 3))


def test_activation_and_inverse_match_oracle():
    n = 3001
    raw = random_raw(n, 1)
    s = empty_surfels(n)
    tr.surfel_activate(cuda(raw), s)
    ref = ot.activate(raw)
    for k in ("mean", "t_u", "t_v", "scale", "opacity", "albedo"):
        np.testing.assert_allclose(to_np(getattr(s, k)), ref[k], rtol=2e-6, atol=2e-6, err_msg=k)
    raw2 = tr.surfel_raw(s)
    s2 = empty_surfels(n)
    tr.surfel_activate(raw2, s2)
    for k in ("mean", "t_u", "t_v", "scale", "opacity", "albedo"):
        np.testing.assert_allclose(to_np(getattr(s2, k)), to_np(getattr(s, k)), atol=5e-6, err_msg=k)


def test_adam_surfels_matches_oracle():
    n, t = 2049, 3
    raw = random_raw(n, 2)
    rng = np.random.default_rng(3)
    m = (rng.standard_normal((n, 13)) * 0.1).astype(np.float32)
    v = (rng.uniform(size=(n, 13)) * 0.01).astype(np.float32)
    g = {k: rng.standard_normal(sh).astype(np.float32) for k, sh in
         (("mean", (n, 3)), ("t_u", (n, 3)), ("t_v", (n, 3)), ("scale", (n, 2)), ("opacity", (n,)),
          ("albedo", (n, 3)))}
    cfg = ot.AdamConfig(lr_mean=0.01, lr_scale=0.003, lr_opacity=0.02, lr_quat=0.004, lr_albedo=0.005,
                        eps=1e-8)
    ccfg = tr.adam_config(lr_mean=0.01, lr_scale=0.003, lr_opacity=0.02, lr_quat=0.004, lr_albedo=0.005,
                          eps=1e-8)
    traw, tm, tv = cuda(raw), cuda(m), cuda(v)
    s = empty_surfels(n)
    tr.adam_surfels(traw, tm, tv, {k: cuda(x) for k, x in g.items()}, ccfg, t, s)
    f32 = lambda x: float(np.float32(x))
    cfg.beta1, cfg.beta2, cfg.eps = f32(0.9), f32(0.999), f32(1e-8)
    graw = ot.activation_adjoint(raw.astype(np.float64), {k: x.astype(np.float64) for k, x in g.items()})
    lr = np.array([f32(x) for x in ot.group_lr(cfg)])
    r1, m1, v1 = ot.adam(raw.astype(np.float64), m.astype(np.float64), v.astype(np.float64), graw,
                         lr, t, cfg)
    np.testing.assert_allclose(to_np(tm), m1, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(to_np(tv), v1, rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(to_np(traw), r1, rtol=1e-5, atol=2e-6)
    ref = ot.activate(to_np(traw))
    for k in ("t_u", "scale", "opacity"):
        np.testing.assert_allclose(to_np(getattr(s, k)), ref[k], rtol=2e-6, atol=2e-6, err_msg=k)


def test_adam_views_camera_start_and_colour():
    nv = 3
    rng = np.random.default_rng(4)
    P = {k: rng.standard_normal(sh).astype(np.float32) for k, sh in
         (("dF", (nv, 2, 4)), ("colC", (nv, 3, 3)), ("colc", (nv, 3)))}
    G = {k: rng.standard_normal(x.shape).astype(np.float32) for k, x in P.items()}
    extra = rng.standard_normal((nv, 2, 4)).astype(np.float32)
    views = ss.ViewTensors(np.full(nv, 4, np.int32), np.full(nv, 4, np.int32), cuda(np.zeros((nv, 2, 4))),
                           1.0, cuda(P["dF"]), cuda(P["colC"]), cuda(P["colc"]))
    state = {}
    for k in P:
        state["m_" + k] = torch.zeros(P[k].shape, dtype=torch.float32, device="cuda")
        state["v_" + k] = torch.zeros(P[k].shape, dtype=torch.float32, device="cuda")
    cfg = tr.adam_config(lr_dF=0.002, lr_colour=0.003, eps=1e-8, camera_start=3)
    grads = {k: cuda(x) for k, x in G.items()}
    for step in (1, 2):   # before the camera start: only the colour terms move
        tr.adam_views(views, state, grads, cfg, step, cuda(extra))
    np.testing.assert_array_equal(to_np(views.dF), P["dF"])
    assert float(state["m_dF"].abs().max()) == 0.0
    oc = ot.AdamConfig(eps=float(np.float32(1e-8)))
    oc.beta1, oc.beta2 = float(np.float32(0.9)), float(np.float32(0.999))
    th, m, v = P["colC"].astype(np.float64), 0.0, 0.0
    for step in (1, 2):
        th, m, v = ot.adam(th, m, v, G["colC"].astype(np.float64), float(np.float32(0.003)), step, oc)
    np.testing.assert_allclose(to_np(views.colC), th, rtol=1e-5, atol=1e-6)
    tr.adam_views(views, state, grads, cfg, 3, cuda(extra))
    # the camera group's first step: -lr sign(g + extra)
    np.testing.assert_allclose(to_np(views.dF), P["dF"] - np.float32(0.002) * np.sign(G["dF"] + extra),
                               rtol=1e-5, atol=1e-6)


def test_l1_loss_matches_oracle():
    sc = synth.make_scene(synth.tiny(n_surfels=50, views=((31, 17), (12, 29)), seed=3))
    plan, surf, views = make_plan(sc)
    P = views.pixels
    rng = np.random.default_rng(5)
    img = rng.uniform(size=3 * P).astype(np.float32)
    tgt = img + rng.choice([-1, 1], 3 * P) * rng.uniform(0.01, 0.2, 3 * P).astype(np.float32)
    d = torch.empty(3 * P, dtype=torch.float32, device="cuda")
    loss = tr.image_loss_l1(plan, cuda(img), cuda(tgt), 0.8, d)
    rl, rg = ot.l1_loss(img, tgt, sc["width"], sc["height"], 0.8)
    np.testing.assert_allclose(to_np(loss), rl, rtol=1e-5)
    np.testing.assert_allclose(to_np(d), rg, rtol=1e-6)


def test_training_step_matches_oracle_and_descends():
    sc = synth.make_scene(synth.tiny(n_surfels=500, views=((36, 31), (30, 34)), seed=24))
    ds = float(np.float32(2.0 / sc["spec"].extent))
    plan, surf, views = make_plan(sc, ts=8)
    first = plan.forward(surf, views)
    P = views.pixels
    rng = np.random.default_rng(6)
    noise = rng.choice([-1, 1], 3 * P) * rng.uniform(0.02, 0.1, 3 * P)
    tgt = (to_np(first["image"]) + noise).astype(np.float32)
    w = tr.LossWeights()
    cfg = tr.adam_config(lr_mean=0.01, camera_start=1, eps=1e-8)
    trainer = tr.Trainer(plan, surf, views, cuda(tgt), ds, cfg=cfg, weights=w)
    raw0 = to_np(trainer.raw).astype(np.float64)
    act = {k: to_np(getattr(surf, k)) for k in ("mean", "t_u", "t_v", "scale", "opacity", "albedo")}
    l1_0, ln_0 = [t.clone() for t in trainer.step()]   # the trainer reuses its loss buffers
    # oracle chain on the same activated surfels
    osc = dict(sc, surfels=act)
    st = oracle_settings(ts=8)
    st.depth_scale = ds
    ref = oracle.forward(osc, st, with_dist=True)
    assert not ref["ambiguous"].any()
    rl1, gI = ot.l1_loss(ref["image"], tgt, sc["width"], sc["height"], w.l1)
    rln, _, gD, gN, gF = geom.normal_loss(osc, ref["depth"], ref["T"], ref["normal"], tau=w.tau)
    np.testing.assert_allclose(to_np(l1_0), rl1, rtol=1e-4)
    np.testing.assert_allclose(to_np(ln_0), w.normal * rln, rtol=1e-4)
    dd = np.concatenate([np.full(int(a) * int(b), w.distortion / (int(a) * int(b)))
                         for a, b in zip(sc["width"], sc["height"])]).astype(np.float32)
    g = oracle.backward(osc, gI, w.normal * gD, w.normal * gN, st, dDist=dd)
    g["dF"] = g["dF"] + w.normal * gF
    graw = ot.activation_adjoint(raw0, g)
    m_gpu = to_np(trainer.m)
    for name, sl in (("mean", slice(0, 3)), ("scale", slice(3, 5)), ("opacity", slice(5, 6)),
                     ("quat", slice(6, 10)), ("albedo", slice(10, 13))):
        assert rel_err(m_gpu[:, sl], 0.1 * graw[:, sl]) < 1e-3, name
    for k in ("dF", "colC", "colc"):
        assert rel_err(to_np(trainer.vstate["m_" + k]), 0.1 * g[k]) < 1e-3, k
    # descent: fit the render of the same scene with darker albedo
    plan2, surf2, views2 = make_plan(sc, ts=8)
    dark = ss.SurfelTensors(surf2.mean, surf2.t_u, surf2.t_v, surf2.scale, surf2.opacity,
                            (surf2.albedo * 0.7).contiguous())
    target = plan2.forward(dark, views2)["image"].clone()
    trainer2 = tr.Trainer(plan2, surf2, views2, target, ds,
                          cfg=tr.adam_config(lr_mean=0.001, camera_start=1000, eps=1e-8), weights=w)
    losses = [float(trainer2.step()[0].sum()) for _ in range(12)]
    assert losses[-1] < 0.8 * losses[0], losses


def test_trainer_checkpoint_resumes_the_run(tmp_path):
    """Save after 3 steps, run 3 more; a new trainer over fresh tensors loads the file and
    runs the same 3 steps.  The restored state is bit-identical (the activated surfels are
    rewritten from the raw parameters), and the continued run matches up to the gradient
    atomics' summation order.  The camera group starts at step 2, so the resumed steps
    depend on the restored step count."""
    sc = synth.make_scene(synth.tiny(n_surfels=500, views=((36, 31), (30, 34)), seed=24))
    ds = float(np.float32(2.0 / sc["spec"].extent))
    w = tr.LossWeights()
    cfg = tr.adam_config(lr_mean=0.001, camera_start=2, eps=1e-8)
    keys = ("mean", "t_u", "t_v", "scale", "opacity", "albedo")

    def fresh():
        plan, surf, views = make_plan(sc, ts=8)
        return plan, surf, views

    plan, surf, views = fresh()
    dark = ss.SurfelTensors(surf.mean, surf.t_u, surf.t_v, surf.scale, surf.opacity,
                            (surf.albedo * 0.7).contiguous())
    target = plan.forward(dark, views)["image"].clone()
    A = tr.Trainer(plan, surf, views, target, ds, cfg=cfg, weights=w)
    for _ in range(3):
        A.step()
    path = tmp_path / "trainer.npz"
    A.save(path)
    saved = A.state_dict()
    act = {k: to_np(getattr(surf, k)).copy() for k in keys}
    la = [float(A.step()[0].sum()) for _ in range(3)]
    endA = A.state_dict()

    plan_b, surf_b, views_b = fresh()
    B = tr.Trainer(plan_b, surf_b, views_b, target, ds, cfg=cfg, weights=w)
    B.load(path)
    assert B.step_count == 3
    for k, a in B.state_dict().items():
        np.testing.assert_array_equal(a, saved[k], err_msg=k)
    for k in keys:
        np.testing.assert_array_equal(to_np(getattr(surf_b, k)), act[k], err_msg=k)
    lb = [float(B.step()[0].sum()) for _ in range(3)]
    np.testing.assert_allclose(lb, la, rtol=1e-4)
    endB = B.state_dict()
    assert endB["step_count"] == endA["step_count"] == 6
    # in norm: a parameter whose gradient is cancellation noise can take a different
    # (tiny) Adam step in the two runs
    for k in endA:
        if k != "step_count":
            a, b = endB[k].astype(np.float64), endA[k].astype(np.float64)
            assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b), k
    # a checkpoint of another trainer shape is refused
    sc2 = synth.make_scene(synth.tiny(n_surfels=300, views=((36, 31), (30, 34)), seed=24))
    plan_c, surf_c, views_c = make_plan(sc2, ts=8)
    C_ = tr.Trainer(plan_c, surf_c, views_c, target, ds, cfg=cfg, weights=w)
    with pytest.raises(ValueError):
        C_.load(path)
