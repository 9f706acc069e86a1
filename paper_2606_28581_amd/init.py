"""Geometry-aware initialisation on a DSM (Sec. 3.4) over the C ABI (argument marshalling
only; the weights, prefix sum, sampling and frames run in libsatsplat.so)."""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import call
from .raster import SurfelTensors, _ptr, _stream


def dsm_init(z: torch.Tensor, x0: float, y0: float, gsd: float, n: int, seed: int,
             opacity: float = 0.5, albedo: float = 0.5, with_cells: bool = False):
    """z: device [ny, nx] FP32 node heights.  Returns SurfelTensors of n surfels (and the
    chosen cell of each when with_cells)."""
    ny, nx = z.shape
    b = C.c_size_t()
    call("ss_dsm_init_workspace_size", int(nx), int(ny), C.byref(b))
    dev = z.device
    ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=dev)
    f = lambda *s: torch.empty(*s, dtype=torch.float32, device=dev)
    s = SurfelTensors(f(n, 3), f(n, 3), f(n, 3), f(n, 2), f(n), f(n, 3))
    cells = torch.empty(n, dtype=torch.int64, device=dev) if with_cells else None
    call("ss_dsm_init", int(nx), int(ny), _ptr(z), float(x0), float(y0), float(gsd), int(n),
         C.c_uint64(int(seed)), float(opacity), float(albedo), C.c_void_p(ws.data_ptr()),
         ws.numel(), _ptr(s.mean), _ptr(s.t_u), _ptr(s.t_v), _ptr(s.scale), _ptr(s.opacity),
         _ptr(s.albedo), _ptr(cells), _stream())
    return (s, cells) if with_cells else s
