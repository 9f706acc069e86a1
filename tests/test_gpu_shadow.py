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
    half = sc["spec"].extent / 2
    for v in range(nv):
        Bs, bs, zfar = oracle.sun_camera(sc, v, S=S)
        np.testing.assert_allclose(cams[v, :6].reshape(2, 3), Bs, rtol=1e-13)
        np.testing.assert_allclose(cams[v, 6:8], bs, rtol=1e-13, atol=1e-10)
        assert cams[v, 8] == pytest.approx(zfar, rel=1e-14)
        # full sun-view depth map vs brute force: normalised depth (units of the scene
        # half-extent) to max-abs 1e-4 on every texel the oracle does not flag ambiguous
        ty, tx = np.meshgrid(np.arange(S), np.arange(S), indexing="ij")
        tex = np.stack([tx.ravel(), ty.ravel()], 1)
        Dref, amb = oracle.sun_depth(sc, Bs, bs, zfar, tex, st, with_ambiguity=True)
        Dref, amb = Dref.reshape(S, S), amb.reshape(S, S)
        assert amb.mean() < 1e-2
        err = np.abs(to_np(D[v]) - Dref)[~amb] / half
        assert err.max() <= 1e-4, err.max()
        # visibility to max-abs 1e-4 on surfels none of whose 3x3 texels is ambiguous
        vref, vamb = oracle.shadow(sc, v, st, with_ambiguity=True)
        vg = to_np(vis[v])
        assert vamb.mean() < 0.05
        verr = np.abs(vg - vref)[~vamb]
        assert verr.max() <= 1e-4, verr.max()
        assert np.mean((vg >= 0.5) == (vref >= 0.5)) > 0.995
    b = plan.debug_binning(1)
    order = oracle.depth_order(sc["surfels"]["mean"], sc["b_z"])
    np.testing.assert_array_equal(b["order"].astype(np.int64), order)


def test_sun_records_centre_box_and_unstored_fields():
    """Sun-view records: the FP32 hi + lo centre equals the FP64 sun-camera projection and
    the pixel box equals the FP64 support box; the shadow pass stores only a record's
    first 16 floats, so the copy-out reads the other 8 as zero."""
    sc = synth.make_scene(synth.tiny(n_surfels=500, views=((40, 40), (31, 22)), seed=9))
    S, ts = 100, 8
    plan, surf, views = make_plan(sc, ts=ts, S=S, with_sun=True)
    plan.shadow(surf, views)
    rec = plan.debug_binning(1, records=True)["records"]
    st = oracle_settings(ts=ts, S=S)
    for v in range(len(sc["width"])):
        Bs, bs, _ = oracle.sun_camera(sc, v, S=S)
        c, _, pix, _ = oracle.binning(sc, Bs, bs, S, S, ts, st)
        cg = rec[v][:, 2:4].astype(np.float64) + rec[v][:, 4:6].astype(np.float64)
        np.testing.assert_allclose(cg, c, rtol=1e-12, atol=1e-9)
        box = rec[v][:, 0:2].view(np.uint32)
        lo = (box & 0xFFFF).astype(np.uint16).view(np.int16).astype(np.int64)
        hi = (box >> 16).astype(np.uint16).view(np.int16).astype(np.int64)
        live = (pix[:, 0] <= pix[:, 1]) & (pix[:, 2] <= pix[:, 3])
        assert live.sum() > 100
        np.testing.assert_array_equal(lo[live, 0], pix[live, 0])
        np.testing.assert_array_equal(hi[live, 0], pix[live, 1])
        np.testing.assert_array_equal(lo[live, 1], pix[live, 2])
        np.testing.assert_array_equal(hi[live, 1], pix[live, 3])
        assert not rec[v][:, 16:].any()


def test_plain_pass_agrees_with_heightfield_ground_truth():
    """On a city whose surfels follow the DSM closely, every surfel of flat ground or roof
    whose sun visibility is clear of the edge band gets the heightfield ray march's
    decision from the GPU's plain pass (tile 8, 256^2 sun maps)."""
    from shadow_truth import confident_flat
    sc = synth.make_scene(synth.shadow_city(n_boxes=8, seed=5))
    plan, surf, views = make_plan(sc, ts=8, S=256, with_sun=True)
    vis = to_np(plan.shadow(surf, views))
    n = sc["surfels"]["mean"].shape[0]
    sel = np.arange(n)
    dark = 0
    for v in range(len(sc["width"])):
        m, conf = confident_flat(sc, sel, v)
        agree = (vis[v] >= 0.5) == (m < 0)
        dark += int((conf & (m > 0)).sum())
        print(f"[shadow-gt] view {v}: {int(conf.sum())} confident surfels, agreement "
              f"{agree[conf].mean():.5f}", flush=True)
        assert agree[conf].all(), (v, np.flatnonzero(conf & ~agree)[:10])
    assert dark > 1500
