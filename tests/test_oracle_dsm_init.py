"""Pins of the DSM-initialisation oracle (Sec. 3.4 "Area-Weighted Sampling", "Splat
Orientation"): the Philox4x32-10 generator against its published known-answer vectors,
closed forms of the area weight and normal on planes, the sampled frequencies against the
weights, and the cell search against a brute-force scan."""
import numpy as np

from oracle import dsm_init as di


def test_philox4x32_10_known_answers():
    """Known-answer vectors published with the Random123 library for Philox4x32, 10 rounds."""
    cases = [((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
             ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
             ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
              (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1))]
    for c, k, want in cases:
        got = di.philox4x32_10(*c, *k)
        assert tuple(int(x) for x in got) == want


def test_plane_weights_normals_heights_and_frames():
    """z = a x + b y on a grid of spacing g: every cell has area g^2 sqrt(1 + a^2 + b^2) and
    normal (-a, -b, 1) / sqrt(1 + a^2 + b^2); the bilinear height of a sample is on the
    plane; frames are orthonormal with t_u, t_v perpendicular to the normal."""
    g, a, b = 0.5, 0.3, -1.7
    x0, y0 = -8.0, -6.0
    xs = x0 + g * np.arange(33)
    ys = y0 + g * np.arange(25)
    X, Y = np.meshgrid(xs, ys)
    z = (a * X + b * Y).astype(np.float32)
    w, area, n = di.cell_geometry(z, g)
    zf = z.astype(np.float64)
    # slopes from the FP32 nodes (exactly a, b up to the rounding of the inputs)
    sx = (zf[:, 1:] - zf[:, :-1]) / g
    sy = (zf[1:, :] - zf[:-1, :]) / g
    assert np.abs(sx - a).max() < 1e-5 and np.abs(sy - b).max() < 1e-5
    np.testing.assert_allclose(area, g * g * np.sqrt(1 + a * a + b * b), rtol=1e-5)
    np.testing.assert_allclose(n, np.broadcast_to(np.array([-a, -b, 1.0]) / np.sqrt(1 + a * a + b * b),
                                                  n.shape), atol=1e-5)
    assert np.all(np.abs(w - 65536 * np.sqrt(1 + a * a + b * b)) <= 2)
    out = di.dsm_init(z, x0, y0, g, 4000, seed=99)
    p = out["mean"]
    np.testing.assert_allclose(p[:, 2], a * p[:, 0] + b * p[:, 1], atol=1e-5)
    for k in ("t_u", "t_v"):
        np.testing.assert_allclose(np.linalg.norm(out[k], axis=1), 1.0, atol=1e-12)
        assert np.abs(np.sum(out[k] * out["normal"], 1)).max() < 1e-12
    assert np.abs(np.sum(out["t_u"] * out["t_v"], 1)).max() < 1e-12
    # scale: spacing of N samples over the surface area
    surf = (len(xs) - 1) * (len(ys) - 1) * g * g * np.sqrt(1 + a * a + b * b)
    np.testing.assert_allclose(out["scale"][0, 0], np.sqrt(surf / 4000), rtol=1e-4)


def test_sampled_cells_follow_the_area_weights():
    """A DSM with a wall: cells at the wall are steep and large; over 400k samples every
    cell's count is within 5 binomial standard deviations of N w / W."""
    g = 0.5
    z = np.zeros((13, 17), np.float32)
    z[:, 9:] = 6.0
    z[4:8, 2:5] = 1.5
    w, _, _ = di.cell_geometry(z, g)
    N = 400_000
    out = di.dsm_init(z, 0.0, 0.0, g, N, seed=7)
    cnt = np.bincount(out["cell"], minlength=w.size)
    p = w / w.sum()
    sd = np.sqrt(N * p * (1 - p))
    assert np.all(np.abs(cnt - N * p) <= 5 * sd + 1)
    assert w.max() > 5 * w.min()          # the wall cells weigh more


def test_cell_search_matches_brute_force():
    rng = np.random.default_rng(3)
    z = rng.uniform(0, 4, size=(9, 11)).astype(np.float32)
    out = di.dsm_init(z, 1.0, 2.0, 0.5, 3000, seed=12345678901)
    w, _, _ = di.cell_geometry(z, 0.5)
    cdf = np.cumsum(w)
    k = np.arange(3000, dtype=np.uint64)
    zero = np.zeros_like(k)
    r0, r1, _, _ = di.philox4x32_10(k, zero, zero, zero, 12345678901 & 0xFFFFFFFF, 12345678901 >> 32)
    t = ((r1.astype(np.uint64) << np.uint64(32)) | r0.astype(np.uint64)) % np.uint64(cdf[-1])
    brute = np.array([next(c for c in range(cdf.size) if cdf[c] > int(tt)) for tt in t])
    np.testing.assert_array_equal(out["cell"], brute)
