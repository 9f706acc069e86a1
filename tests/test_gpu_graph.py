"""Batched whole-step execution: eager ss_step, HIP-graph replay and the autotuner.

A graph replay must reproduce the eager step exactly (forward outputs bitwise,
gradients up to atomic-order rounding), also after inputs change between replays and
with the program's own eager work and synchronisations in between."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2606_28581_amd as ss
from gpu_common import ATOMIC_ORDER_TOL, GRAD_KEYS, make_plan, oracle_settings, rel_err, to_np

pytestmark = pytest.mark.gpu


def setup(seed=21, S=64, n=500):
    sc = synth.make_scene(synth.tiny(n_surfels=n, views=((47, 41), (30, 52), (64, 64)), seed=seed))
    plan, surf, views = make_plan(sc, S=S, with_sun=True)
    dI, dD, dN = [torch.as_tensor(x, device="cuda") for x in synth.upstream_grads(sc)]
    bufs = ss.StepBuffers(surf.mean.shape[0], views.width, views.height, upstream=(dI, dD, dN),
                          sun_map=S)
    return sc, plan, surf, views, bufs


def snapshot(bufs):
    out = {k: to_np(v).copy() for k, v in bufs.out.items()}
    out["vis_in"] = to_np(bufs.vis).copy()
    g = {k: to_np(v).copy() for k, v in bufs.grads.items()}
    return out, g


def test_eager_step_matches_separate_calls_and_oracle():
    sc, plan, surf, views, bufs = setup()
    ss.step(plan, surf, views, bufs)
    torch.cuda.synchronize()
    out, g = snapshot(bufs)
    vis = plan.shadow(surf, views)
    f = plan.forward(surf, views, vis)
    np.testing.assert_array_equal(to_np(vis), out["vis_in"])
    np.testing.assert_array_equal(to_np(f["image"]), out["image"])
    st = oracle_settings(S=64)
    ref = oracle.forward(sc, st, vis=out["vis_in"])
    ok = ~ref["ambiguous"]
    assert np.abs(out["T"][ok] - ref["T"][ok]).max() < 1e-4


def test_graph_replays_match_eager_across_input_changes():
    sc, plan, surf, views, bufs = setup(seed=22)
    ss.step(plan, surf, views, bufs)
    torch.cuda.synchronize()
    eager_out, eager_g = snapshot(bufs)
    graph = ss.Graph(plan, surf, views, bufs)
    for rep in range(3):
        for t in list(bufs.out.values()) + list(bufs.grads.values()):
            t.zero_()                     # eager work between replays
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        out, g = snapshot(bufs)
        for k in eager_out:
            np.testing.assert_array_equal(out[k], eager_out[k], err_msg=f"replay {rep} {k}")
        for k in GRAD_KEYS:
            assert rel_err(g[k], eager_g[k]) < ATOMIC_ORDER_TOL, (rep, k)
    # change inputs in place; the replay must see them
    with torch.no_grad():
        views.colC.mul_(0.9)
        surf.albedo.mul_(0.8)
    graph.launch()
    torch.cuda.synchronize()
    rep_out, rep_g = snapshot(bufs)
    ss.step(plan, surf, views, bufs)
    torch.cuda.synchronize()
    new_out, new_g = snapshot(bufs)
    np.testing.assert_array_equal(rep_out["image"], new_out["image"])
    assert not np.array_equal(new_out["image"], eager_out["image"])
    for k in GRAD_KEYS:
        assert rel_err(rep_g[k], new_g[k]) < ATOMIC_ORDER_TOL, k
    over, _, _ = plan.check()
    assert not over


def test_autotune_leaves_plan_on_a_candidate_that_keeps_parity():
    sc, plan, surf, views, bufs = setup(seed=23)
    best, ms, table = ss.autotune(plan, surf, views, bufs, reps=2)
    assert best.tile_size in (8, 16, 32) and best.batch_depth in (32, 64, 128, 256)
    ran = table[:, 2] > 0
    assert ms > 0 and ran.sum() == 10                     # batch 128 and 256 exceed 8x8 threads
    assert np.all(table[~ran, 1] > table[~ran, 0] ** 2)
    assert ms == pytest.approx(table[ran, 2].min())
    ss.step(plan, surf, views, bufs)
    torch.cuda.synchronize()
    vis = to_np(bufs.vis)
    ref = oracle.forward(sc, oracle_settings(ts=best.tile_size, S=64), vis=vis)
    ok = ~ref["ambiguous"]
    ok3 = np.concatenate([np.tile(ok[o:o + w * h], 3) for o, w, h in
                          zip(np.cumsum([0] + [w * h for w, h in zip(sc["width"], sc["height"])])[:-1],
                              sc["width"], sc["height"])])
    assert np.abs(to_np(bufs.out["image"])[ok3] - ref["image"][ok3]).max() < 1e-4
