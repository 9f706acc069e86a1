"""Heightfield ground truth of sun visibility for the shadow-pass tests (CPU and GPU)."""
import numpy as np

from oracle import heightfield as hf


def confident_flat(sc, sel, v, margin=0.5, start=2.0, band=2):
    """Ground-truth margin of the selected surfels and the mask of the confident ones:
    flat ground or roof (every DSM height within 1 m equals the point's own), the
    decision at least `margin` metres of altitude from changing, and unchanged when the
    DSM is grown (lit points) or shrunk (shadowed points) sideways by `band` nodes --
    the edge band where a surfel reaching past a roof's edge may move the shadow (a
    surfel reaches 3.3 scales, 1 m for the 0.3 m surfels, two nodes at 0.5 m GSD)."""
    coords, z = sc["dsm"]
    mean = sc["surfels"]["mean"].astype(np.float64)[sel]
    phi, theta = (float(a) for a in sc["sun"][v])
    m = hf.sun_margin(coords, z, mean, phi, theta, start=start)
    grown = hf.sun_margin(coords, hf.window_filter(z, band, np.maximum), mean, phi, theta, start=start)
    shrunk = hf.sun_margin(coords, hf.window_filter(z, band, np.minimum), mean, phi, theta, start=start)
    g = float(coords[1] - coords[0])
    flat = np.ones(len(sel), bool)
    for dx in (-1.0, 0.0, 1.0):
        for dy in (-1.0, 0.0, 1.0):
            hh = hf.bilinear(coords, z, mean[:, 0] + dx, mean[:, 1] + dy)
            flat &= np.abs(hh - mean[:, 2]) < 0.05 * g
    lit = (m < -margin) & (grown < -margin)
    dark = (m > margin) & (shrunk > margin)
    return m, flat & (lit | dark)
