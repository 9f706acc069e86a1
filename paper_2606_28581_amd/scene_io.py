"""Move a seeded synthetic scene (numpy arrays) to device tensors."""
from __future__ import annotations

import numpy as np
import torch

from .raster import SurfelTensors, ViewTensors


def scene_to_device(scene, device="cuda:0", with_sun=None):
    t = lambda a: None if a is None else torch.as_tensor(np.ascontiguousarray(a, np.float32),
                                                          device=device)
    s = scene["surfels"]
    surf = SurfelTensors(t(s["mean"]), t(s["t_u"]), t(s["t_v"]), t(s["scale"]),
                         t(s["opacity"]), t(s["albedo"]))
    sun = scene.get("sun") if with_sun is None or with_sun else None
    views = ViewTensors(np.asarray(scene["width"], np.int32), np.asarray(scene["height"], np.int32),
                        t(scene["Fxy"]), float(scene["b_z"]), t(scene.get("dF")),
                        t(scene.get("colC")), t(scene.get("colc")), t(scene.get("ambient")),
                        t(sun))
    return surf, views
