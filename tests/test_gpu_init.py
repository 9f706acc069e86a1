"""GPU parity of the geometry-aware DSM initialisation (Sec. 3.4; HIP kernels through the
C ABI) against the FP64 oracle: the chosen cells bit-exact (the weights are integers and
the decisions are taken on them), centres, frames and scales to FP32 rounding; at the
5M-surfel scale on the 2 x 2 km city DSM, on a sample of the surfels."""
import numpy as np
import pytest
import torch

import synth
from synth.scene import _streams, make_dsm
from oracle import dsm_init as odi
from paper_2606_28581_amd import init as gi
from gpu_common import to_np

pytestmark = pytest.mark.gpu


def dsm_of(spec):
    coords, z = make_dsm(spec, _streams(spec.seed)["scene"])
    return float(coords[0]), float(spec.gsd), z.astype(np.float32)


def check(s, cells, ref, rows=None):
    pick = (lambda t: to_np(t)) if rows is None else (lambda t: to_np(t)[rows])
    np.testing.assert_array_equal(pick(cells), ref["cell"])
    np.testing.assert_allclose(pick(s.mean), ref["mean"], rtol=0, atol=2e-4)
    np.testing.assert_allclose(pick(s.t_u), ref["t_u"], atol=2e-6)
    np.testing.assert_allclose(pick(s.t_v), ref["t_v"], atol=2e-6)
    np.testing.assert_allclose(pick(s.scale), ref["scale"], rtol=2e-7)
    np.testing.assert_array_equal(pick(s.opacity), ref["opacity"].astype(np.float32))
    np.testing.assert_array_equal(pick(s.albedo), ref["albedo"].astype(np.float32))


@pytest.mark.parametrize("n", [1, 777, 50_000])
def test_dsm_init_small_city_matches_oracle(n):
    spec = synth.tiny(n_surfels=10, extent=40.0, n_boxes=5, seed=4)
    x0, g, z = dsm_of(spec)
    s, cells = gi.dsm_init(torch.as_tensor(z, device="cuda"), x0, x0, g, n, seed=0xDEADBEEF12,
                           opacity=0.3, albedo=0.6, with_cells=True)
    ref = odi.dsm_init(z, x0, x0, g, n, seed=0xDEADBEEF12, opacity=0.3, albedo=0.6)
    check(s, cells, ref)


def test_dsm_init_5m_surfels_on_the_2km_city():
    spec = synth.config(5)
    x0, g, z = dsm_of(spec)
    n = spec.n_surfels
    s, cells = gi.dsm_init(torch.as_tensor(z, device="cuda"), x0, x0, g, n, seed=2024,
                           with_cells=True)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(1).choice(n, 4000, replace=False))
    rows = np.concatenate([rows, [0, n - 1]])
    ref = odi.dsm_init(z, x0, x0, g, n, seed=2024, sel=rows)
    check(s, cells, ref, rows)
    # every surfel lies on the DSM surface's footprint and its frame is orthonormal
    m = to_np(s.mean)
    half = spec.extent / 2
    assert m[:, 0].min() >= -half and m[:, 0].max() <= half
    tu, tv = to_np(s.t_u), to_np(s.t_v)
    assert np.abs(np.linalg.norm(tu, axis=1) - 1).max() < 1e-5
    assert np.abs(np.sum(tu * tv, 1)).max() < 1e-5
