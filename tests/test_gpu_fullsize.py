"""Parity at full size, in the launch configuration the benchmark times (tile 8, batch
depth 64), on sampled outputs that the FP64 oracle computes one by one, plus properties
that hold at every pixel.

* 2M surfels, 40 views of sides 1024..2048 px, 1024^2 sun maps: 512 pixels over 8 views,
  half of them drawn from the 1 % longest 8x8 tile lists (where multi-word contributor
  masks and long back-to-front walks run); their image, albedo, visibility, depth,
  normal, transmittance and every gradient they cause.  The sun pass is checked on a
  sample of surfels, visibility to max-abs 1e-4 where none of a surfel's 3x3 sun-map
  texels is threshold-ambiguous.
* 1M surfels, one 2048^2 view with camera delta and colour correction, and 5M surfels
  on the 2x2 km city, one 2048^2 view: sampled pixels and their gradients.

Visibility enters the forward as a seeded per-(view, surfel) input on both sides; the
oracle renders each sampled pixel by brute force over all surfels.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2606_28581_amd as ss
from gpu_common import context, oracle_settings, rel_err, to_np

pytestmark = pytest.mark.gpu

T_MIN = np.float32(1e-4)
TS = 8


def support_rel_err(a, b):
    """rel_err over the entries either side sets (the gradients of a few hundred sampled
    pixels touch a small part of the surfels; the rms floor is taken over those)."""
    a = np.asarray(a, np.float64).reshape(-1)
    b = np.asarray(b, np.float64).reshape(-1)
    s = (a != 0) | (b != 0)
    return rel_err(a[s], b[s]) if s.any() else 0.0


def sub_scene(sc, vs):
    pick = lambda a: None if a is None else a[list(vs)]
    return dict(sc, width=sc["width"][list(vs)], height=sc["height"][list(vs)],
                Fxy=pick(sc["Fxy"]), dF=pick(sc["dF"]), colC=pick(sc["colC"]),
                colc=pick(sc["colc"]), ambient=pick(sc["ambient"]), sun=pick(sc["sun"]))


def tile_lengths(sc, v, ost):
    """Pairs per 8x8 tile of view v from the oracle's FP64 binning (2D difference array
    over each surfel's tile rectangle)."""
    W, H = int(sc["width"][v]), int(sc["height"][v])
    B, b = oracle.view_camera(sc, v)
    _, _, _, tiles = oracle.binning(sc, B, b, W, H, TS, ost)
    tx, ty = (W + TS - 1) // TS, (H + TS - 1) // TS
    live = tiles[:, 0] <= tiles[:, 1]
    t = tiles[live].astype(np.int64)
    d = np.zeros((ty + 1, tx + 1), np.int64)
    np.add.at(d, (t[:, 2], t[:, 0]), 1)
    np.add.at(d, (t[:, 2], t[:, 1] + 1), -1)
    np.add.at(d, (t[:, 3] + 1, t[:, 0]), -1)
    np.add.at(d, (t[:, 3] + 1, t[:, 1] + 1), 1)
    return np.cumsum(np.cumsum(d, 0), 1)[:ty, :tx]


def pick_pixels(sc, views, per_view, long_frac, rng, ost):
    """Per view: per_view * (1 - long_frac) uniform pixels and the rest inside the 1 %
    longest tiles.  Returns local pixel indices per view."""
    out = []
    for v in views:
        W, H = int(sc["width"][v]), int(sc["height"][v])
        n_long = int(per_view * long_frac)
        uni = rng.choice(W * H, per_view - n_long, replace=False)
        picks = list(uni)
        if n_long:
            L = tile_lengths(sc, v, ost)
            cut = np.quantile(L, 0.99)
            ty, tx = np.nonzero(L >= cut)
            k = rng.choice(ty.size, n_long, replace=True)
            for a, c in zip(tx[k], ty[k]):
                i = min(W - 1, a * TS + int(rng.integers(TS)))
                j = min(H - 1, c * TS + int(rng.integers(TS)))
                picks.append(j * W + i)
        out.append(np.unique(np.asarray(picks, np.int64)))
    return out


def n_views_str(sc):
    return f"{sc['spec'].n_surfels} surfels, {len(sc['width'])} views"


class Workload:
    def __init__(self, sc, views, per_view, long_frac, seed, with_sun=False):
        self.sc = sc
        self.views = tuple(views)
        surf, vt = ss.scene_to_device(sc, with_sun=with_sun)
        st = ss.default_settings(tile_size=TS, batch_depth=64)
        self.plan = ss.Plan(context(), surf.mean.shape[0], vt.width, vt.height, st)
        self.plan.ensure_capacity(surf, vt)
        self.surf, self.vt = surf, vt
        self.ost = oracle_settings(ts=TS, S=1024)
        self.sub = sub_scene(sc, self.views)
        rng = np.random.default_rng(seed)
        local = pick_pixels(sc, self.views, per_view, long_frac, rng, self.ost)
        self.off_all = synth.pixel_offsets(sc["width"], sc["height"])
        off_sub = synth.pixel_offsets(self.sub["width"], self.sub["height"])
        print(f"[fullsize] {n_views_str(sc)}: plan sized, pixels picked", flush=True)
        self.sel_all = np.concatenate([self.off_all[v] + l for v, l in zip(self.views, local)])
        self.sel_sub = np.concatenate([off_sub[k] + l for k, l in enumerate(local)])
        n, nv = surf.mean.shape[0], len(sc["width"])
        self.vis = rng.uniform(0.0, 1.0, size=(nv, n)).astype(np.float32)
        self.vis_sub = self.vis[list(self.views)]
        W, H = sc["width"], sc["height"]
        rows = []
        for g in self.sel_all:
            v = int(np.searchsorted(self.off_all, g, side="right") - 1)
            P, loc = int(W[v]) * int(H[v]), int(g - self.off_all[v])
            rows.append([3 * self.off_all[v] + ch * P + loc for ch in range(3)])
        self.rows = np.asarray(rows)
        self.out = None
        self.ref = None

    def forward(self):
        vis = torch.as_tensor(self.vis, device="cuda")
        out = self.plan.forward(self.surf, self.vt, vis)
        self.out = out
        self.ref = oracle.forward(self.sub, self.ost, vis=self.vis_sub, sel=self.sel_sub)
        print(f"[fullsize] forward of {len(self.sel_all)} pixels: GPU and oracle done", flush=True)
        return {k: to_np(t) for k, t in out.items()}

    def check_forward(self, o):
        ref, rows, sel = self.ref, self.rows, self.sel_all
        ok = ~ref["ambiguous"]
        assert ok.mean() > 0.99
        half = self.sc["spec"].extent / 2
        np.testing.assert_allclose(o["image"][rows][ok], ref["image"].reshape(-1, 3)[ok], atol=1e-4)
        np.testing.assert_allclose(o["albedo"][rows][ok], ref["albedo"].reshape(-1, 3)[ok], atol=1e-4)
        np.testing.assert_allclose(o["normal"][rows][ok], ref["normal"].reshape(-1, 3)[ok], atol=1e-4)
        np.testing.assert_allclose(o["vis"][sel][ok], ref["vis"][ok], atol=1e-4)
        np.testing.assert_allclose(o["T"][sel][ok], ref["T"][ok], atol=1e-4)
        np.testing.assert_allclose(o["depth"][sel][ok] / half, ref["depth"][ok] / half, atol=1e-4)
        return ok

    def check_backward(self, ok, seed):
        g = np.random.default_rng(seed)
        m, rows, sel = len(self.sel_all), self.rows, self.sel_all
        dI_c = (g.standard_normal((m, 3)) * ok[:, None]).astype(np.float32)
        dD_c = (g.standard_normal(m) * ok).astype(np.float32)
        dN_c = (g.standard_normal((m, 3)) * ok[:, None]).astype(np.float32)
        P_all = int(self.off_all[-1])
        dI = np.zeros(3 * P_all, np.float32); dN = np.zeros(3 * P_all, np.float32)
        dD = np.zeros(P_all, np.float32)
        dI[rows.ravel()] = dI_c.ravel(); dN[rows.ravel()] = dN_c.ravel(); dD[sel] = dD_c
        cu = lambda a: torch.as_tensor(a, device="cuda")
        gg = self.plan.backward(self.surf, self.vt, self.out, cu(dI), cu(dD), cu(dN),
                                vis=cu(self.vis))
        gr = oracle.backward(self.sub, dI_c.ravel(), dD_c, dN_c.ravel(), self.ost,
                             vis=self.vis_sub, sel=self.sel_sub)
        print(f"[fullsize] backward of {m} pixels: GPU and oracle done", flush=True)
        for key in ("mean", "t_u", "t_v", "scale", "opacity", "albedo"):
            assert np.abs(gr[key]).max() > 0, key
            assert support_rel_err(to_np(gg[key]), gr[key]) < 1e-3, key
        nv = len(self.sc["width"])
        for key in ("dF", "colC", "colc", "ambient"):
            gv = to_np(gg[key])
            assert rel_err(gv[list(self.views)], gr[key]) < 1e-3, key
            others = np.setdiff1d(np.arange(nv), self.views)
            if others.size:
                assert np.abs(gv[others]).max() == 0.0, key


C3_VIEWS = (0, 5, 10, 15, 20, 25, 30, 39)


@pytest.fixture(scope="module")
def c3():
    sc = synth.make_scene(synth.config(3))
    return Workload(sc, C3_VIEWS, per_view=64, long_frac=0.5, seed=77, with_sun=True)


def test_c3_forward_sampled_pixels_and_every_pixel_properties(c3):
    o = c3.forward()
    for key in ("image", "albedo", "vis", "depth", "normal", "T"):
        assert np.all(np.isfinite(o[key])), key
    assert o["T"].min() >= T_MIN and o["T"].max() <= 1.0
    assert len(c3.sel_all) >= 500
    c3.ok = c3.check_forward(o)


def test_c3_backward_sampled_pixels(c3):
    if c3.out is None:
        pytest.skip("needs the forward test's outputs")
    c3.check_backward(c3.ok, seed=78)


def test_c3_sun_pass_on_sampled_surfels(c3):
    vis = to_np(c3.plan.shadow(c3.surf, c3.vt))
    rng = np.random.default_rng(79)
    n = c3.surf.mean.shape[0]
    for v in (0, 39):
        sel = np.sort(rng.choice(n, 96, replace=False))
        one = sub_scene(c3.sc, (v,))
        vref, amb = oracle.shadow(one, 0, c3.ost, sel=sel, with_ambiguity=True)
        vg = vis[v, sel]
        assert amb.mean() < 0.1
        err = np.abs(vg - vref)[~amb]
        assert err.max() <= 1e-4, (v, err.max())


def test_c3_sun_pass_against_heightfield_ground_truth(c3):
    """Agreement of the plain pass with the heightfield ray march on the 1 km city, on a
    sample of flat-ground and roof surfels clear of the edge band.  The city's surfels
    (scales up to 2 m, opacity sigmoid(N(0, 1))) reach metres past the roof edges, so
    this is a measurement of the scene against its DSM rather than a parity bound."""
    from shadow_truth import confident_flat
    vis = to_np(c3.plan.shadow(c3.surf, c3.vt))
    n = c3.surf.mean.shape[0]
    sel = np.sort(np.random.default_rng(81).choice(n, 20000, replace=False))
    for v in (0, 39):
        m, conf = confident_flat(c3.sc, sel, v, band=4)
        agree = (vis[v, sel] >= 0.5) == (m < 0)
        lit, dark = conf & (m < 0), conf & (m > 0)
        print(f"[fullsize] c3 view {v}: heightfield agreement {agree[conf].mean():.4f} over "
              f"{int(conf.sum())} surfels (lit {agree[lit].mean():.4f}, shadowed "
              f"{agree[dark].mean():.4f} of {int(dark.sum())})", flush=True)
        assert conf.sum() > 3000 and dark.sum() > 100
        assert agree[conf].mean() > 0.99


@pytest.mark.parametrize("cfg", [2, 5])
def test_single_view_sampled_pixels(cfg):
    """1M surfels on the 1 km city and 5M on the 2 km city, one 2048^2 view each."""
    spec = synth.config(cfg, views=[(2048, 2048)]) if cfg == 5 else synth.config(cfg)
    sc = synth.make_scene(spec)
    w = Workload(sc, (0,), per_view=96, long_frac=0.5, seed=80 + cfg)
    o = w.forward()
    assert np.all(np.isfinite(o["image"])) and o["T"].min() >= T_MIN
    ok = w.check_forward(o)
    w.check_backward(ok, seed=90 + cfg)
