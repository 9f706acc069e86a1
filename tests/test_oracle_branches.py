"""Pins of the oracle's alpha_max clamp and degenerate-surfel branches.

The clamp alpha = min(alpha_max, o G) (reading of Eq. rasterization, where the adjoint
gives zero gradient to o and G above alpha_max) and the degenerate branch of Sec. 3.2
"Degenerate Solutions" (no uv branch, low-pass disk only) are pinned by
  * behaviour: switching the clamp or the degenerate test off changes the render, so the
    scene reaches both branches;
  * an independent second statement of the definition (dense torch FP64, autograd)
    agreeing with the C oracle's forward and analytic adjoint;
  * FP64 central differences of the forward on entries whose step does not cross any
    discrete decision (the per-pixel decision digest is the same at x - h, x and x + h).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from branch_scenes import branch_scene, special_surfels
from oracle import Settings, dense


@pytest.mark.parametrize("mode", [0, 1])
def test_branch_scene_reaches_clamp_and_degenerate_branches(mode):
    sc = branch_scene()
    base = oracle.forward(sc, Settings(lowpass_mode=mode))
    noclamp = oracle.forward(sc, Settings(lowpass_mode=mode, alpha_max=np.float32(0.99999).item()))
    assert np.abs(base["image"] - noclamp["image"]).max() > 1e-3
    # coverage of the degenerate test: |det T| <= 1e-6 |T|_F^2 for the edge-on surfels in
    # the view they face, and det T == 0 exactly for vertical t_v in the exact-nadir view
    s = sc["surfels"]
    _, deg = special_surfels(sc)
    n_deg, n_zero = 0, 0
    for v in range(len(sc["width"])):
        F = sc["Fxy"][v].astype(np.float64) + sc["dF"][v].astype(np.float64)
        for k in deg:
            M = np.stack([s["scale"][k, 0] * s["t_u"][k].astype(np.float64),
                          s["scale"][k, 1] * s["t_v"][k].astype(np.float64)], axis=1)
            T = F[:, :3] @ M
            det = T[0, 0] * T[1, 1] - T[0, 1] * T[1, 0]
            n_deg += abs(det) <= 1e-6 * np.sum(T * T)
            n_zero += det == 0.0
    assert n_deg >= len(deg) and n_zero >= 8
    if mode == 1:
        # without the degenerate test an edge-on splat has no low-pass floor in mode 1:
        # the render changes
        nodeg = oracle.forward(sc, Settings(lowpass_mode=mode, det_rel_eps=0.0))
        assert np.abs(base["image"] - nodeg["image"]).max() > 1e-3
    assert base["ambiguous"].mean() < 0.02


@pytest.mark.parametrize("mode,with_vis", [(0, True), (1, False), (1, True)])
def test_branch_scene_c_oracle_matches_dense_torch(mode, with_vis):
    sc = branch_scene()
    n = sc["surfels"]["mean"].shape[0]
    V = len(sc["width"])
    st = Settings(lowpass_mode=mode)
    vis = np.random.default_rng(4).uniform(size=(V, n)).astype(np.float32) if with_vis else None
    out = oracle.forward(sc, st, vis=vis)
    P = dense.params_from_scene(sc)
    r = dense.render(P, sc, st, vis=vis)
    cat = lambda k: torch.cat([x[k].reshape(-1) for x in r])
    ok = ~out["ambiguous"]
    for k in ("image", "albedo", "normal"):
        np.testing.assert_allclose(cat(k).detach().numpy(), out[k], atol=1e-12)
    for k in ("depth", "T", "vis"):
        np.testing.assert_allclose(cat(k).detach().numpy()[ok], out[k][ok], atol=1e-11)
    dI, dD, dN = synth.upstream_grads(sc)
    L = (cat("image") * torch.as_tensor(dI, dtype=torch.float64)).sum() + \
        (cat("depth") * torch.as_tensor(dD, dtype=torch.float64)).sum() + \
        (cat("normal") * torch.as_tensor(dN, dtype=torch.float64)).sum()
    L.backward()
    g = oracle.backward(sc, dI, dD, dN, st, vis=vis)
    clamp, deg = special_surfels(sc)
    for k in ("mean", "t_u", "t_v", "scale", "opacity", "albedo", "dF", "colC", "colc", "ambient"):
        a = P[k].grad.numpy().reshape(-1)
        b = g[k].reshape(-1)
        scale = max(np.abs(a).max(), 1e-30)
        assert np.abs(a - b).max() <= 1e-11 * scale, k
    # the special surfels receive gradient (they are composited)
    assert np.abs(g["mean"][deg]).max() > 0 and np.abs(g["albedo"][clamp]).max() > 0


def _loss(sc, dI, dD, dN, vis, st):
    out = oracle.forward(sc, st, vis=vis)
    order = oracle.depth_order(sc["surfels"]["mean"], sc["b_z"])
    return out["image"] @ dI + out["depth"] @ dD + out["normal"] @ dN, \
        np.concatenate([out["sig"].view(np.int64), order])


@pytest.mark.parametrize("mode", [0, 1])
def test_branch_scene_adjoint_matches_central_differences(mode):
    sc = branch_scene()
    n = sc["surfels"]["mean"].shape[0]
    V = len(sc["width"])
    rng = np.random.default_rng(17 + mode)
    vis = rng.uniform(size=(V, n)).astype(np.float32)
    dI, dD, dN = [x.astype(np.float64) for x in synth.upstream_grads(sc)]
    st = Settings(lowpass_mode=mode)
    g = oracle.backward(sc, dI, dD, dN, st, vis=vis)
    _, k0 = _loss(sc, dI, dD, dN, vis, st)
    clamp, deg = special_surfels(sc)
    special = np.concatenate([clamp, deg])
    groups = [("mean", sc["surfels"], 3), ("t_u", sc["surfels"], 3), ("t_v", sc["surfels"], 3),
              ("scale", sc["surfels"], 2), ("opacity", sc["surfels"], 1),
              ("albedo", sc["surfels"], 3), ("dF", sc, 0)]
    checked, checked_special = 0, 0
    for name, holder, width in groups:
        arr = holder[name]
        flat = arr.reshape(-1)
        gg = g[name].reshape(-1)
        rms = np.sqrt(np.mean(gg ** 2)) + 1e-30
        if width:
            pool = (special[:, None] * width + np.arange(width)[None]).reshape(-1)
            idx = np.concatenate([rng.choice(pool, size=min(14, pool.size), replace=False),
                                  rng.choice(flat.size, size=6, replace=False)])
        else:
            idx = rng.choice(flat.size, size=min(12, flat.size), replace=False)
        for i in idx:
            x0 = flat[i]
            h = np.float32(max(1.0, abs(float(x0))) * 1e-5)
            xp, xm = np.float32(x0 + h), np.float32(x0 - h)
            flat[i] = xp
            lp, kp = _loss(sc, dI, dD, dN, vis, st)
            flat[i] = xm
            lm, km = _loss(sc, dI, dD, dN, vis, st)
            flat[i] = x0
            if not (np.array_equal(kp, k0) and np.array_equal(km, k0)):
                continue   # a discrete decision (skip, stop, branch, clamp, flag, flip) moved
            fd = (lp - lm) / (np.float64(xp) - np.float64(xm))
            err = abs(fd - gg[i]) / max(abs(gg[i]), 1e-2 * rms)
            assert err < 1e-5, (name, i, fd, gg[i])
            checked += 1
            if width and i // width in special:
                checked_special += 1
    print("checked", checked, checked_special)
    assert checked > 70 and checked_special > 40, (checked, checked_special)
