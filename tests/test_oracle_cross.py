"""Two independent statements of the same definition agree: the C oracle (per-pixel
loop, analytic adjoint) and the dense torch-FP64 version (all pairs at once, autograd)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import Settings, dense


@pytest.mark.parametrize("mode,with_vis", [(0, True), (1, False)])
def test_c_oracle_matches_dense_torch_forward_and_gradients(mode, with_vis):
    sc = synth.make_scene(synth.tiny(n_surfels=260, views=((31, 27), (22, 35)), seed=21))
    st = Settings(lowpass_mode=mode)
    vis = None
    if with_vis:
        vis = np.random.default_rng(9).uniform(size=(2, 260)).astype(np.float32)
    out = oracle.forward(sc, st, vis=vis)
    P = dense.params_from_scene(sc)
    r = dense.render(P, sc, st, vis=vis)
    cat = lambda k: torch.cat([x[k].reshape(-1) for x in r])
    ok = ~out["ambiguous"]
    for k in ("image", "albedo", "normal"):
        a, b = cat(k).detach().numpy().reshape(-1), out[k]
        np.testing.assert_allclose(a, b, atol=1e-12)
    for k in ("depth", "T", "vis"):
        np.testing.assert_allclose(cat(k).detach().numpy()[ok], out[k][ok], atol=1e-11)
    dI, dD, dN = synth.upstream_grads(sc)
    L = (cat("image") * torch.as_tensor(dI, dtype=torch.float64)).sum() + \
        (cat("depth") * torch.as_tensor(dD, dtype=torch.float64)).sum() + \
        (cat("normal") * torch.as_tensor(dN, dtype=torch.float64)).sum()
    L.backward()
    g = oracle.backward(sc, dI, dD, dN, st, vis=vis)
    for k in ("mean", "t_u", "t_v", "scale", "opacity", "albedo", "dF", "colC", "colc", "ambient"):
        a = P[k].grad.numpy().reshape(-1)
        b = g[k].reshape(-1)
        scale = max(np.abs(a).max(), 1e-30)
        assert np.abs(a - b).max() <= 1e-11 * scale, k
