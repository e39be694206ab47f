"""ctypes declarations of the isogs C ABI (include/isogs.h).

Argument marshalling only: every computation runs in libisogs.so.  Importing
this module loads the in-tree library and fails loudly when it has not been
built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libisogs.so")

GS_OK = 0
GS_ERR = {
    -1: "GS_ERR_INVALID", -2: "GS_ERR_NOMEM", -3: "GS_ERR_HIP", -4: "GS_ERR_CAPACITY",
    -5: "GS_ERR_UNSUPPORTED", -6: "GS_ERR_BUSY",
}

EXPORT = {"keys": 0, "values": 1, "ranges": 2, "final_T": 3, "n_contrib": 4,
          "screen_grads": 5, "splats": 6, "rects": 7, "depths": 8}


class IsogsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{GS_ERR.get(status, status)}: {msg}")
        self.status = status


class GsParams(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("n", C.c_int64),
                ("sh_degree", C.c_int32), ("reserved", C.c_int32)]


class GsCamera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("z_near", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("reserved", C.c_int32)]


class GsRenderOpts(C.Structure):
    _fields_ = [("tile", C.c_int32), ("lds_depth", C.c_int32), ("bg", C.c_float * 3),
                ("flags", C.c_int32)]


class GsAdamOpts(C.Structure):
    _fields_ = [("lr_means", C.c_float), ("lr_log_scales", C.c_float), ("lr_quats", C.c_float),
                ("lr_opacity", C.c_float), ("lr_sh_dc", C.c_float), ("lr_sh_rest", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("zero_grads", C.c_int32)]


class GsInitOpts(C.Structure):
    _fields_ = [("log_scale", C.c_float), ("log_scale_jitter", C.c_float),
                ("log_scale_lo", C.c_float), ("log_scale_hi", C.c_float),
                ("random_quats", C.c_int32), ("opacity_logit", C.c_float),
                ("sh_std", C.c_float), ("reserved", C.c_int32)]


class GsFrameStats(C.Structure):
    _fields_ = [("n_views", C.c_int32), ("tile", C.c_int32), ("n_gaussians", C.c_int64),
                ("n_records", C.c_int64), ("n_visible", C.c_int64), ("n_tiles", C.c_int64),
                ("n_pixels", C.c_int64), ("device_bytes", C.c_int64)]


_P = C.c_void_p
_PP = C.POINTER(C.c_void_p)


class GsStepDesc(C.Structure):
    _fields_ = [("params", GsParams), ("grads", GsParams), ("adam_m", GsParams),
                ("adam_v", GsParams), ("cams", C.POINTER(GsCamera)), ("n_views", C.c_int32),
                ("images", _PP), ("targets", _PP), ("dl_dimg", _PP), ("loss", _P),
                ("render", GsRenderOpts), ("adam", GsAdamOpts), ("with_adam", C.c_int32),
                ("lambda_dssim", C.c_float), ("first_step", C.c_int64),
                ("capacity_slack", C.c_double)]


class GsServerOpts(C.Structure):
    _fields_ = [("n_slots", C.c_int32), ("max_batch_views", C.c_int32),
                ("mem_budget", C.c_size_t), ("render", GsRenderOpts), ("max_queue", C.c_int32),
                ("reserved", C.c_int32)]


class GsServeStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("batches", C.c_int64),
                ("deferred", C.c_int64), ("mean_batch_views", C.c_double),
                ("p50_ms", C.c_double), ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("max_ms", C.c_double), ("mpix_per_s", C.c_double), ("peak_bytes", C.c_int64)]


class GsDensityStats(C.Structure):
    _fields_ = [("grad", C.c_void_p), ("count", C.c_void_p), ("max_radius", C.c_void_p),
                ("n", C.c_int64)]


class GsDensityOpts(C.Structure):
    _fields_ = [("grad_threshold", C.c_double), ("percent_dense", C.c_double),
                ("min_opacity", C.c_double), ("max_screen", C.c_double),
                ("max_world", C.c_double), ("extent", C.c_double), ("split_div", C.c_double),
                ("n_split", C.c_int32), ("reserved", C.c_int32), ("seed", C.c_uint64)]


class GsDensityInfo(C.Structure):
    _fields_ = [("n_in", C.c_int64), ("n_out", C.c_int64), ("kept", C.c_int64),
                ("cloned", C.c_int64), ("split", C.c_int64), ("children", C.c_int64),
                ("pruned", C.c_int64)]


class GsVolume(C.Structure):
    _fields_ = [("values", C.c_void_p), ("nx", C.c_int64), ("ny", C.c_int64), ("nz", C.c_int64),
                ("lo", C.c_float * 3), ("hi", C.c_float * 3)]


class GsTuneEntry(C.Structure):
    _fields_ = [("tile", C.c_int32), ("lds_depth", C.c_int32), ("flags", C.c_int32),
                ("ms", C.c_float)]

# (name, restype, argtypes)
SIGNATURES = [
    ("gs_last_error", C.c_char_p, []),
    ("gs_version", C.c_char_p, []),
    ("gs_ctx_create", C.c_int, [C.c_int, C.c_size_t, C.POINTER(_P)]),
    ("gs_ctx_destroy", None, [_P]),
    ("gs_ctx_memory", C.c_int, [_P, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    ("gs_ctx_set_timing", C.c_int, [_P, C.c_int32]),
    ("gs_ctx_stage_time", C.c_int, [_P, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_int64)]),
    ("gs_stage_name", C.c_char_p, [C.c_int32]),
    ("gs_orbit_cameras", C.c_int, [C.c_int32, C.c_float, C.c_float, C.c_int32, C.c_int32,
                                   C.POINTER(GsCamera)]),
    ("gs_init_from_points", C.c_int, [_P, _P, C.c_int64, C.POINTER(GsInitOpts), C.c_uint64,
                                      GsParams, _P]),
    ("gs_render_fwd", C.c_int, [_P, GsParams, C.POINTER(GsCamera), C.c_int32, _PP,
                                C.POINTER(GsRenderOpts), C.POINTER(_P), _P]),
    ("gs_render_fwd_multi", C.c_int, [_P, C.POINTER(GsParams), C.POINTER(GsCamera), C.c_int32,
                                      _PP, C.POINTER(GsRenderOpts), C.POINTER(_P), _P]),
    ("gs_loss_grad", C.c_int, [_P, _PP, _PP, C.POINTER(GsCamera), C.c_int32, C.c_float, _P,
                               _PP, _P]),
    ("gs_loss_grad_noalloc", C.c_int, [_P, _PP, _PP, C.POINTER(GsCamera), C.c_int32,
                                       C.c_float, _P, _PP, _P]),
    ("gs_image_metrics", C.c_int, [_P, _PP, _PP, C.POINTER(GsCamera), C.c_int32, _P, _P]),
    ("gs_render_bwd", C.c_int, [_P, _P, GsParams, _PP, GsParams, C.c_int32, _P]),
    ("gs_density_accumulate", C.c_int, [_P, _P, GsDensityStats, C.c_float, _P]),
    ("gs_densify", C.c_int, [_P, GsParams, GsParams, GsParams, GsDensityStats,
                             C.POINTER(GsDensityOpts), GsParams, GsParams, GsParams, _P,
                             C.POINTER(GsDensityInfo), _P]),
    ("gs_opacity_reset", C.c_int, [_P, GsParams, GsParams, GsParams, C.c_double, _P]),
    ("gs_iso_extract", C.c_int, [_P, GsVolume, C.c_float, C.c_float, C.c_uint64, _P, C.c_int64,
                                 C.POINTER(C.c_int64), _P]),
    ("gs_raycast", C.c_int, [_P, GsVolume, C.c_float, C.POINTER(GsCamera), C.c_int32,
                             C.c_float, _PP, _P]),
    ("gs_adam_step", C.c_int, [_P, GsParams, GsParams, GsParams, GsParams,
                               C.POINTER(GsAdamOpts), C.c_int64, _P]),
    ("gs_bw_probe", C.c_int, [_P, _P, _P, C.c_size_t, _P]),
    ("gs_frame_stats_get", C.c_int, [_P, C.POINTER(GsFrameStats)]),
    ("gs_frame_export", C.c_int, [_P, C.c_int32, C.c_int32, _P, C.c_size_t, _P]),
    ("gs_frame_release", None, [_P]),
    ("gs_step_graph_create", C.c_int, [_P, C.POINTER(GsStepDesc), C.POINTER(_P), _P]),
    ("gs_step_graph_capture", C.c_int, [_P, C.POINTER(GsStepDesc), C.POINTER(_P)]),
    ("gs_step_graph_launch", C.c_int, [_P, _P]),
    ("gs_step_graph_sync", C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int64), _P]),
    ("gs_step_graph_run", C.c_int, [_P, C.POINTER(C.c_int64), _P]),
    ("gs_step_graph_info", C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                     C.POINTER(_P)]),
    ("gs_step_graph_destroy", None, [_P]),
    ("gs_server_create", C.c_int, [_P, C.POINTER(GsServerOpts), C.POINTER(_P)]),
    ("gs_server_add_scene", C.c_int, [_P, GsParams, C.POINTER(C.c_int32)]),
    ("gs_server_submit", C.c_int, [_P, C.c_int32, C.POINTER(GsCamera), _P,
                                   C.POINTER(C.c_uint64)]),
    ("gs_server_poll", C.c_int, [_P, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("gs_server_wait", C.c_int, [_P, C.c_uint64, C.POINTER(C.c_double)]),
    ("gs_server_drain", C.c_int, [_P]),
    ("gs_server_stats", C.c_int, [_P, C.POINTER(GsServeStats)]),
    ("gs_server_reset_stats", C.c_int, [_P]),
    ("gs_server_destroy", None, [_P]),
    ("gs_autotune", C.c_int, [_P, GsParams, C.POINTER(GsCamera), C.c_int32, C.c_int32,
                              C.POINTER(GsRenderOpts), C.POINTER(GsTuneEntry), C.c_int32,
                              C.POINTER(C.c_int32), _P]),
]

_lib = None


def lib():
    """The loaded library (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != GS_OK:
        raise IsogsError(status, lib().gs_last_error().decode(errors="replace"))


def ptr_array(ptrs):
    arr = (C.c_void_p * len(ptrs))(*ptrs)
    return C.cast(arr, _PP), arr
