"""ctypes declarations of the C ABI in include/satsplat.h (argument marshalling only).

Every step of the hot path runs in libsatsplat.so; nothing here computes.  Loading
fails loudly when the library has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsatsplat.so")

SS_OK = 0
SS_ERR_INVALID_ARG = -1
SS_ERR_CAPACITY = -2
SS_ERR_HIP = -3
SS_ERR_UNSUPPORTED = -4
SS_ERR_STATE = -5


class RasterSettings(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("tile_size", C.c_int32),
                ("batch_depth", C.c_int32), ("alpha_min", C.c_float),
                ("alpha_max", C.c_float), ("T_min", C.c_float), ("lowpass_sigma", C.c_float),
                ("lowpass_mode", C.c_int32), ("det_rel_eps", C.c_float), ("esm_c", C.c_float),
                ("esm_bias", C.c_float), ("sun_map_size", C.c_int32),
                ("tile_order", C.c_int32)]


class Surfels(C.Structure):
    _fields_ = [("n", C.c_int64), ("mean", C.c_void_p), ("t_u", C.c_void_p),
                ("t_v", C.c_void_p), ("scale", C.c_void_p), ("opacity", C.c_void_p),
                ("albedo", C.c_void_p)]


class Views(C.Structure):
    _fields_ = [("n", C.c_int32), ("width", C.POINTER(C.c_int32)),
                ("height", C.POINTER(C.c_int32)), ("Fxy", C.c_void_p), ("dF", C.c_void_p),
                ("colC", C.c_void_p), ("colc", C.c_void_p), ("ambient", C.c_void_p),
                ("sun", C.c_void_p), ("b_z", C.c_float)]


class StepIO(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("vis", C.c_void_p), ("sun_depth", C.c_void_p),
                ("image", C.c_void_p), ("albedo_out", C.c_void_p), ("vis_out", C.c_void_p),
                ("depth", C.c_void_p), ("normal", C.c_void_p), ("T_final", C.c_void_p),
                ("last", C.c_void_p), ("d_image", C.c_void_p), ("d_depth", C.c_void_p),
                ("d_normal", C.c_void_p), ("d_mean", C.c_void_p), ("d_t_u", C.c_void_p),
                ("d_t_v", C.c_void_p), ("d_scale", C.c_void_p), ("d_opacity", C.c_void_p),
                ("d_albedo", C.c_void_p), ("d_dF", C.c_void_p), ("d_colC", C.c_void_p),
                ("d_colc", C.c_void_p), ("d_ambient", C.c_void_p)]


class GeomIO(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("depth_scale", C.c_float), ("dist", C.c_void_p),
                ("aux", C.c_void_p), ("d_dist", C.c_void_p)]


class AdamConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("lr_mean", C.c_float), ("lr_scale", C.c_float),
                ("lr_opacity", C.c_float), ("lr_quat", C.c_float), ("lr_albedo", C.c_float),
                ("lr_dF", C.c_float), ("lr_colour", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("camera_start", C.c_int32)]


class MlpConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("centre", C.c_float * 3), ("inv_half", C.c_float)]


_P = C.c_void_p
_I64P = C.POINTER(C.c_int64)
_SIGS = {
    "ss_last_error": (C.c_char_p, []),
    "ss_default_settings": (None, [C.POINTER(RasterSettings)]),
    "ss_context_create": (C.c_int32, [C.c_int32, C.POINTER(_P)]),
    "ss_context_destroy": (C.c_int32, [_P]),
    "ss_plan_create": (C.c_int32, [_P, C.c_int64, C.c_int32, C.POINTER(C.c_int32),
                                   C.POINTER(C.c_int32), C.POINTER(RasterSettings),
                                   C.POINTER(_P)]),
    "ss_plan_destroy": (C.c_int32, [_P]),
    "ss_plan_set_settings": (C.c_int32, [_P, C.POINTER(RasterSettings)]),
    "ss_plan_workspace_size": (C.c_int32, [_P, C.c_int64, C.c_int64, C.POINTER(C.c_size_t)]),
    "ss_plan_bind_workspace": (C.c_int32, [_P, _P, C.c_size_t, C.c_int64, C.c_int64]),
    "ss_count_pairs": (C.c_int32, [_P, C.POINTER(Surfels), C.POINTER(Views), _I64P, _I64P, _P]),
    "ss_plan_check": (C.c_int32, [_P, C.POINTER(C.c_int32), _I64P, _I64P, _P]),
    "ss_forward": (C.c_int32, [_P, C.POINTER(Surfels), C.POINTER(Views), _P, _P, _P, _P, _P,
                               _P, _P, _P, _P]),
    "ss_backward": (C.c_int32, [_P, C.POINTER(Surfels), C.POINTER(Views), _P, _P, _P, _P, _P,
                                _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ss_forward_geom": (C.c_int32, [_P, C.POINTER(Surfels), C.POINTER(Views), _P, _P, _P, _P,
                                    _P, _P, _P, _P, C.POINTER(GeomIO), _P]),
    "ss_backward_geom": (C.c_int32, [_P, C.POINTER(Surfels), C.POINTER(Views), _P, _P, _P, _P,
                                     _P, _P, _P, _P, C.POINTER(GeomIO), _P, _P, _P, _P, _P, _P,
                                     _P, _P, _P, _P, _P]),
    "ss_normal_loss": (C.c_int32, [_P, C.POINTER(Views), _P, _P, _P, C.c_float, C.c_float, _P,
                                   _P, _P, _P, _P, _P]),
    "ss_surfel_activate": (C.c_int32, [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ss_dsm_init_workspace_size": (C.c_int32, [C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "ss_dsm_init": (C.c_int32, [C.c_int32, C.c_int32, _P, C.c_float, C.c_float, C.c_float, C.c_int64,
                                C.c_uint64, C.c_float, C.c_float, _P, C.c_size_t, _P, _P, _P, _P, _P,
                                _P, _P, _P]),
    "ss_surfel_raw": (C.c_int32, [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P]),
    "ss_adam_surfels": (C.c_int32, [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                    C.POINTER(AdamConfig), C.c_int32, _P, _P, _P, _P, _P, _P, _P]),
    "ss_adam_views": (C.c_int32, [C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                  C.POINTER(AdamConfig), C.c_int32, _P]),
    "ss_image_loss_l1": (C.c_int32, [_P, _P, _P, C.c_float, _P, _P, _P]),
    "ss_shadow_plain": (C.c_int32, [_P, C.POINTER(Surfels), C.POINTER(Views), _P, _P, _P]),
    "ss_debug_binning": (C.c_int32, [_P, C.c_int32, _P, _P, _P, _P, _P, _I64P, _I64P, _P]),
    "ss_debug_sun_cameras": (C.c_int32, [_P, _P, _P]),
    "ss_plan_set_timing": (C.c_int32, [_P, C.c_int32]),
    "ss_plan_read_timing": (C.c_int32, [_P, _P, _P]),
    "ss_stage_name": (C.c_char_p, [C.c_int32]),
    "ss_plan_stats": (C.c_int32, [_P, _P, _P]),
    "ss_step": (C.c_int32, [_P, C.POINTER(Surfels), C.POINTER(Views), C.POINTER(StepIO), _P]),
    "ss_graph_build": (C.c_int32, [_P, C.POINTER(Surfels), C.POINTER(Views), C.POINTER(StepIO),
                                   C.POINTER(_P)]),
    "ss_graph_launch": (C.c_int32, [_P, _P]),
    "ss_graph_destroy": (C.c_int32, [_P]),
    "ss_autotune": (C.c_int32, [_P, C.POINTER(Surfels), C.POINTER(Views), C.POINTER(StepIO),
                                C.c_int32, C.POINTER(RasterSettings), C.POINTER(C.c_double),
                                _P, _P]),
    "ss_mlp_create": (C.c_int32, [_P, C.POINTER(MlpConfig), C.POINTER(_P)]),
    "ss_mlp_destroy": (C.c_int32, [_P]),
    "ss_mlp_workspace_size": (C.c_int32, [_P, C.c_int64, C.POINTER(C.c_size_t)]),
    "ss_mlp_bind_workspace": (C.c_int32, [_P, _P, C.c_size_t, C.c_int64]),
    "ss_mlp_forward": (C.c_int32, [_P, _P, _P, C.c_int64, _P, C.c_int64, C.c_int32, C.c_int32,
                                   _P, _P]),
    "ss_mlp_backward": (C.c_int32, [_P, _P, _P, _P, C.c_int64, _P, _P, C.c_float, _P, _P, _P]),
    "ss_mlp_backward_noalloc": (C.c_int32, [_P, _P, _P, _P, C.c_int64, _P, _P, C.c_float, _P, _P,
                                            _P]),
    "ss_mlp_adam": (C.c_int32, [_P, _P, _P, _P, C.c_int64, C.c_float, C.c_float, C.c_float,
                                C.c_float, C.c_int32, _P]),
    "ss_shadow_surrogate": (C.c_int32, [_P, _P, _P, C.POINTER(Surfels), C.POINTER(Views),
                                        C.c_float, _P, _P, _P]),
}

SS_NUM_STAGES = 16
SS_RAW_FLOATS = 13
SS_MLP_PARAMS = 16641
SS_NOALLOC_MAX_POINTS = 16384

_lib = None


class SatSplatError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


def load():
    """Load libsatsplat.so (built in-tree by __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def call(name, *args):
    """Call an ss_* entry point; raise SatSplatError on a negative status."""
    lib = load()
    st = getattr(lib, name)(*args)
    if st is not None and st != SS_OK:
        raise SatSplatError(name, st, lib.ss_last_error().decode())
    return st


def declared_functions(header_path):
    """Names of the functions declared in a public header (for the export test)."""
    import re
    text = open(header_path).read()
    return sorted(set(re.findall(r"\b(ss_[a-z_]+)\s*\(", text)))


# Aliases with the C names, for callers who prefer the flat ABI.
def __getattr__(name):
    if name.startswith("ss_"):
        lib = load()
        return getattr(lib, name)
    raise AttributeError(name)
