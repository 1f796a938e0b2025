"""ctypes declarations of libgs4d.so (the C ABI of include/gs4d.h)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgs4d.so")

GS_OK = 0
GS_ERR_INVALID_ARG = -1
GS_ERR_WORKSPACE = -2
GS_ERR_PAIR_OVERFLOW = -3
GS_ERR_HIP = -4
GS_ERR_NO_DEVICE = -5
GS_ERR_UNSUPPORTED = -6


class GsSettings(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
        ("n_levels", ctypes.c_int32), ("level_counts", ctypes.c_int32 * 8), ("level_weights", ctypes.c_float * 8),
        ("res_channels", ctypes.c_int32), ("near_plane", ctypes.c_float), ("dilation", ctypes.c_float),
        ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float), ("t_stop", ctypes.c_float),
        ("bg", ctypes.c_float * 3), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
        ("bin_chunk", ctypes.c_int32), ("row_seg", ctypes.c_int32), ("wave_layout", ctypes.c_int32),
        ("lds_batch", ctypes.c_int32), ("bwd_pixels", ctypes.c_int32),
    ]


class GsWorkspaceLayout(ctypes.Structure):
    _fields_ = [(k, ctypes.c_size_t) for k in (
        "status", "records", "rects", "keys", "vals", "ranges", "lists", "t_final", "n_last", "grad2d",
        "composed", "total")] + [("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                                 ("pair_capacity", ctypes.c_int64)]


class GsStats(ctypes.Structure):
    _fields_ = [("overflow", ctypes.c_int32), ("pad", ctypes.c_int32)] + [
        (k, ctypes.c_int64) for k in ("needed_pairs", "fwd_evals", "fwd_contribs", "bwd_evals", "bwd_contribs")]


class GsRateDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_attr", ctypes.c_int32), ("step", ctypes.c_float), ("mode", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("offset", ctypes.c_uint64), ("n_levels", ctypes.c_int32),
        ("level_counts", ctypes.c_int32 * 8), ("level_weights", ctypes.c_float * 8), ("lambda_rate", ctypes.c_float),
        ("fit_scale", ctypes.c_float), ("blocks_per_attr", ctypes.c_int32), ("offset_dev", ctypes.c_void_p),
    ]


class GsMapsLayout(ctypes.Structure):
    _fields_ = [
        ("n_channels", ctypes.c_int32), ("n_levels", ctypes.c_int32), ("level_counts", ctypes.c_int32 * 8),
        ("width", ctypes.c_int32 * 8), ("height", ctypes.c_int32 * 8), ("offset", ctypes.c_int64 * 8),
        ("total_bytes", ctypes.c_int64),
    ]


class GsEntropyDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_attr", ctypes.c_int32), ("step", ctypes.c_float), ("mode", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("offset", ctypes.c_uint64), ("n_levels", ctypes.c_int32),
        ("level_counts", ctypes.c_int32 * 8), ("level_weights", ctypes.c_float * 8), ("lambda_rate", ctypes.c_float),
        ("kind", ctypes.c_int32), ("lambda_reg", ctypes.c_float),
    ]


class GsMotionDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("box_lo", ctypes.c_float * 3), ("box_hi", ctypes.c_float * 3)]


_lib = None

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
SZ = ctypes.c_size_t

SIGNATURES = {
    "gs_workspace_size": ([P, I32, I32, I32, I64, P], ctypes.c_int),
    "gs_workspace_describe": ([P, I32, I32, I32, I64, P], ctypes.c_int),
    "gs_render_forward": ([P, I32, P, I32, P, I32, P, P, P, SZ, P], ctypes.c_int),
    "gs_render_backward": ([P, I32, P, I32, P, I32, P, P, P, P, P, P, P, P, SZ, P], ctypes.c_int),
    "gs_check_status": ([P, P, P], ctypes.c_int),
    "gs_autotune_render": ([P, I32, P, I32, P, I32, P, P, P, P, P, SZ, P, P, P], ctypes.c_int),
    "gs_color_loss_workspace_size": ([P, I32, I32, P], ctypes.c_int),
    "gs_color_loss": ([P, I32, I32, P, P, ctypes.c_float, P, P, P, SZ, P], ctypes.c_int),
    "gs_significance_workspace_size": ([I32, P], ctypes.c_int),
    "gs_significance_order": ([I32, P, I32, ctypes.c_float, P, P, P, SZ, P], ctypes.c_int),
    "gs_maps_describe": ([I32, I32, P, P], ctypes.c_int),
    "gs_encode_workspace_size": ([P, P], ctypes.c_int),
    "gs_encode_maps": ([P, P, P, P, P, P, P, SZ, P], ctypes.c_int),
    "gs_decode_maps": ([P, P, P, P, P], ctypes.c_int),
    "gs_entropy_workspace_size": ([P, P], ctypes.c_int),
    "gs_entropy_model": ([P, P, P, P, P, P, P, SZ, P], ctypes.c_int),
    "gs_motion_sizes": ([P, P], ctypes.c_int),
    "gs_motion_workspace_size": ([I32, P], ctypes.c_int),
    "gs_motion_forward": ([P, P, I32, P, P, P, P], ctypes.c_int),
    "gs_motion_backward": ([P, P, I32, P, P, P, P, P, P, SZ, P], ctypes.c_int),
    "gs_error_string": ([ctypes.c_int], ctypes.c_char_p),
    "gs_last_error": ([], ctypes.c_char_p),
    "gs_workspace_stats": ([P, P, P], ctypes.c_int),
    "gs_set_work_counters": ([ctypes.c_int], ctypes.c_int),
    "gs_set_deterministic": ([ctypes.c_int], ctypes.c_int),
    "gs_zero": ([P, SZ, P], ctypes.c_int),
    "gs_profile_enable": ([ctypes.c_int], ctypes.c_int),
    "gs_profile_collect": ([I32, P, P], ctypes.c_int),
    "gs_kernel_name": ([I32], ctypes.c_char_p),
    "gs_rate_histogram_workspace_size": ([I32, P], ctypes.c_int),
    "gs_rate_model": ([P, P, P, P, P, P, P, P, P, P, P, P], ctypes.c_int),
    "gs_rate_autotune": ([P, P, P, P, P, P, P, P, P, P, P, P], ctypes.c_int),
    "gs_rate_histogram": ([I32, I32, P, ctypes.c_float, P, P, SZ, P], ctypes.c_int),
    "gs_rate_init_output_bias": ([I32, I32, P, ctypes.c_float, P, P, P], ctypes.c_int),
    "gs_peak_fma": ([I32, I32, ctypes.c_float, ctypes.c_float, P, P], ctypes.c_int),
    "gs_adam_step_dev": ([I64, P, P, P, P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P, P],
                         ctypes.c_int),
    "gs_advance_counters": ([P, P, ctypes.c_uint64, P], ctypes.c_int),
    "gs_peak_copy": ([P, P, SZ, P], ctypes.c_int),
    "gs_rate_histogram_noalloc": ([I32, I32, P, ctypes.c_float, P, P], ctypes.c_int),
    "gs_rate_context": ([I32, P, ctypes.c_float, I32, P, P, P], ctypes.c_int),
    "gs_adam_step": ([I64, P, P, P, P, P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                      I32, P], ctypes.c_int),
}


class GsError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        msg = L.gs_error_string(code).decode()
        detail = L.gs_last_error().decode()
        super().__init__(f"{where}: {msg} ({code}){': ' + detail if detail else ''}")
        self.code = code


def lib():
    """Loads the HIP library; raises if it has not been built (there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`"
                              " or `python paper_2509_17513_amd/build.py`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
        _lib = L
    return _lib


def check(code: int, where: str):
    if code != GS_OK:
        raise GsError(code, where)
