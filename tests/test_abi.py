"""Host-side checks of the C ABI (no GPU needed): the library loads and exports every
entry point include/satsplat.h declares; defaults match the documented readings;
argument validation fails cleanly without touching a device."""
import ctypes as C
import os

import numpy as np
import pytest
import torch

import paper_2606_28581_amd as ss
from paper_2606_28581_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "satsplat.h")


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _lib.declared_functions(HEADER)
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib._SIGS, f"{name} has no ctypes signature"


def test_struct_layouts_match_header():
    assert C.sizeof(_lib.RasterSettings) == 4 * 13
    assert C.sizeof(_lib.Surfels) == 8 * 7
    assert C.sizeof(_lib.Views) == 8 * 10


def test_default_settings_are_the_documented_readings():
    s = ss.default_settings()
    assert s.struct_size == C.sizeof(_lib.RasterSettings)
    assert s.tile_size == 16
    assert s.alpha_min == pytest.approx(1 / 255)
    assert s.alpha_max == pytest.approx(0.99)
    assert s.T_min == pytest.approx(1e-4)
    assert s.lowpass_sigma == pytest.approx(0.70710678)
    assert s.sun_map_size == 1024
    assert s.tile_order == 0


def test_invalid_arguments_fail_without_a_device():
    lib = _lib.load()
    out = C.c_void_p()
    s = ss.default_settings()
    w = (C.c_int32 * 1)(16)
    st = lib.ss_plan_create(None, 10, 1, w, w, C.byref(s), C.byref(out))
    assert st == _lib.SS_ERR_INVALID_ARG
    assert b"context" in lib.ss_last_error()
    assert lib.ss_forward(None, None, None, None, None, None, None, None, None, None, None,
                          None) == _lib.SS_ERR_INVALID_ARG
    sz = C.c_size_t()
    assert lib.ss_plan_workspace_size(None, 0, 0, C.byref(sz)) == _lib.SS_ERR_INVALID_ARG


@pytest.mark.skipif(torch.cuda.is_available(), reason="checks the no-device error path")
def test_context_without_gpu_reports_hip_error():
    with pytest.raises(ss.SatSplatError) as e:
        ss.Context(0)
    assert e.value.code in (_lib.SS_ERR_HIP, _lib.SS_ERR_INVALID_ARG)
