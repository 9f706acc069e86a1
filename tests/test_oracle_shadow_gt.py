"""The geometric shadow pass against ground truth that does not come from shadow maps
(Sec. 3.1 shadow-mapping note, Sec. 3.3 sun camera, Supp. A): sun visibility by
marching the ray towards the sun over the DSM heightfield (`oracle/heightfield.py`).

The march is pinned first against the closed form of one box on flat ground (shadow
length h / tan theta).  The oracle's plain pass is then compared with it on a city whose
surfels follow the DSM closely (0.3 m, opacity 0.95), on points of flat ground whose
decision is at least 1 m of altitude away from changing; the march starts 2 m from the
point, beyond the reach of the point's own surfel (3.3 scales)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import Settings
from oracle import heightfield as hf
from shadow_truth import confident_flat


def box_dsm(h, box, g=0.25, half=16.0):
    coords = -half + g * np.arange(int(round(2 * half / g)) + 1)
    X, Y = np.meshgrid(coords, coords)
    x0, x1, y0, y1 = box
    z = np.where((X >= x0) & (X <= x1) & (Y >= y0) & (Y <= y1), h, 0.0)
    return coords, z


def box_closed_form(q, h, phi, theta, box):
    """Shadowed iff the ground segment from q towards the sun, of length h / tan theta,
    enters the footprint (a segment-rectangle test by the slab method)."""
    x0, x1, y0, y1 = box
    L = h / math.tan(theta)
    d = (L * math.cos(phi), L * math.sin(phi))
    lo, hi = 0.0, 1.0
    for p, dd, a, b in ((q[0], d[0], x0, x1), (q[1], d[1], y0, y1)):
        if abs(dd) < 1e-15:
            if p < a or p > b:
                return False
            continue
        t0, t1 = (a - p) / dd, (b - p) / dd
        lo, hi = max(lo, min(t0, t1)), min(hi, max(t0, t1))
    return lo <= hi


@pytest.mark.parametrize("phi_deg,theta_deg", [(30.0, 45.0), (200.0, 35.0), (300.0, 62.0)])
def test_heightfield_march_matches_box_closed_form(phi_deg, theta_deg):
    h, box = 7.0, (-3.0, 3.0, -2.0, 2.5)
    phi, theta = math.radians(phi_deg), math.radians(theta_deg)
    coords, z = box_dsm(h, box)
    rng = np.random.default_rng(int(phi_deg))
    q = rng.uniform(-15, 15, size=(4000, 2))
    outside = ~((q[:, 0] >= box[0] - 0.5) & (q[:, 0] <= box[1] + 0.5) &
                (q[:, 1] >= box[2] - 0.5) & (q[:, 1] <= box[3] + 0.5))
    q = q[outside]
    # the march starts 1 m out: a lit point's margin is then at least tan(theta) m
    m = hf.sun_margin(coords, z, np.c_[q, np.zeros(len(q))], phi, theta, start=1.0)
    expect = np.array([box_closed_form(p, h, phi, theta, box) for p in q])
    # the bilinear DSM ramps from h to 0 over one node spacing outside the footprint:
    # keep rays whose decision is the same for the footprint grown by that ramp, and
    # points whose decision is not within 0.3 m of altitude of changing
    g = 0.25
    grown = (box[0] - g, box[1] + g, box[2] - g, box[3] + g)
    same = np.array([box_closed_form(p, h, phi, theta, grown) for p in q]) == expect
    clear = same & (np.abs(m) > 0.3)
    assert clear.mean() > 0.8 and expect[clear].sum() > 50
    np.testing.assert_array_equal(m[clear] > 0, expect[clear])
    # the margin is exact on the shadow's far side: altitude left to climb
    ok = (m > 0.3) & (m < h - 0.3)
    assert ok.sum() > 20


def test_window_filter_grows_and_shrinks_a_box():
    z = np.zeros((9, 9))
    z[3:6, 2:7] = 4.0
    g = hf.window_filter(z, 1, np.maximum)
    s = hf.window_filter(z, 1, np.minimum)
    assert np.array_equal(g > 0, np.pad(np.ones((5, 7), bool), ((2, 2), (1, 1))))
    assert np.array_equal(s > 0, np.pad(np.ones((1, 3), bool), ((4, 4), (3, 3))))


def test_plain_pass_agrees_with_heightfield_ground_truth():
    """Every confident surfel's plain-pass decision (v >= 0.5) is the ground truth's."""
    sc = synth.make_scene(synth.shadow_city(n_boxes=8, seed=5))
    n = sc["surfels"]["mean"].shape[0]
    sel = np.sort(np.random.default_rng(1).choice(n, 3000, replace=False))
    lit_total = shadow_total = 0
    for v in range(len(sc["width"])):
        vis = oracle.shadow(sc, v, Settings(sun_map_size=256), sel=sel)
        m, conf = confident_flat(sc, sel, v)
        agree = (vis >= 0.5) == (m < 0)
        lit_total += int((conf & (m < 0)).sum())
        shadow_total += int((conf & (m > 0)).sum())
        assert agree[conf].all(), (v, np.flatnonzero(conf & ~agree))
    assert lit_total > 2500 and shadow_total > 150
