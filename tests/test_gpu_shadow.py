"""GPU parity of the sun-view shadow pass against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_common import make_plan, oracle_settings, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("S,ts", [(64, 16), (100, 8)])
def test_sun_cameras_depth_maps_and_visibility(S, ts):
    sc = synth.make_scene(synth.tiny(n_surfels=500, views=((40, 40), (31, 22)), seed=9))
    plan, surf, views = make_plan(sc, ts=ts, S=S, with_sun=True)
    nv = len(sc["width"])
    D = torch.empty(nv, S, S, device="cuda")
    vis = plan.shadow(surf, views, sun_depth=D)
    cams = plan.debug_sun_cameras()
    st = oracle_settings(ts=ts, S=S)
    for v in range(nv):
        Bs, bs, zfar = oracle.sun_camera(sc, v, S=S)
        np.testing.assert_allclose(cams[v, :6].reshape(2, 3), Bs, rtol=1e-13)
        np.testing.assert_allclose(cams[v, 6:8], bs, rtol=1e-13, atol=1e-10)
        assert cams[v, 8] == pytest.approx(zfar, rel=1e-14)
        # full sun-view depth map vs brute force
        ty, tx = np.meshgrid(np.arange(S), np.arange(S), indexing="ij")
        tex = np.stack([tx.ravel(), ty.ravel()], 1)
        Dref = oracle.sun_depth(sc, Bs, bs, zfar, tex, st).reshape(S, S)
        err = np.abs(to_np(D[v]) - Dref)
        assert np.quantile(err, 0.999) < 1e-3 and err.max() < 0.5, err.max()
        vref = oracle.shadow(sc, v, st)
        vg = to_np(vis[v])
        assert np.abs(vg - vref).max() < 1e-2 or np.mean(np.abs(vg - vref) < 1e-3) > 0.99
        assert np.mean((vg >= 0.5) == (vref >= 0.5)) > 0.995
    b = plan.debug_binning(1)
    order = oracle.depth_order(sc["surfels"]["mean"], sc["b_z"])
    np.testing.assert_array_equal(b["order"].astype(np.int64), order)
