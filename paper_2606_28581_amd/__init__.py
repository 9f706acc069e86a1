"""MI355X (gfx950) hot path of SatSplat (arXiv 2606.28581): the affine-camera 2D
Gaussian surfel rasterizer (forward + hand-written backward) and the geometric sun-view
shadow pass, as hand-written HIP kernels behind the C ABI in include/satsplat.h.

PyTorch supplies device memory and streams only.  There is no CPU fallback: if
libsatsplat.so is missing, loading raises.
"""
from ._lib import SatSplatError, load  # noqa: F401
from .raster import (Context, Graph, Plan, RasterizeAffine2DGS, StepBuffers,  # noqa: F401
                     SurfelTensors, ViewTensors, autotune, default_settings, rasterize, step)
from .scene_io import scene_to_device  # noqa: F401
