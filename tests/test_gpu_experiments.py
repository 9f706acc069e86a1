"""The synthetic camera-robustness experiment (Sec. 4 "Camera Optimization Robustness")
end to end on the GPU: camera errors injected in normalised coordinates are reduced by
gradient descent on the camera deltas through the library's L1 loss, backward and Adam;
with no error injected the descent stays at the true camera."""
import numpy as np
import pytest

import synth
from paper_2606_28581_amd import experiments
from gpu_common import context

pytestmark = pytest.mark.gpu


def test_camera_robustness_recovers_injected_errors():
    sc = synth.make_scene(synth.tiny(n_surfels=3000, views=((72, 64), (64, 70), (68, 68)), extent=40.0,
                                     n_boxes=4, seed=12))
    rows = experiments.camera_robustness(sc, magnitudes=(1e-2, 4e-2), steps=150, ctx=context(),
                                         log=print)
    for r in rows:
        assert r["l1_after"] < r["l1_before"], r
        assert r["ratio"] < 0.5, r
