"""ctypes declarations of the C ABI in include/gsparc.h and the library loader.

The product path has no fallback: if libgsparc.so is missing or fails to load,
``lib()`` raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsparc.so")

c_f32 = ctypes.c_float
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_u32 = ctypes.c_uint32
c_sz = ctypes.c_size_t
c_p = ctypes.c_void_p

GS_OK, GS_ERR_INVALID_ARG, GS_ERR_WORKSPACE, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_NONFINITE = range(6)


class GsScene(ctypes.Structure):
    _fields_ = [("n", c_i32), ("mean", c_p), ("log_scale", c_p), ("quat", c_p), ("opacity_logit", c_p)]


class GsDensifyParams(ctypes.Structure):
    _fields_ = [("grad_threshold", c_f32), ("clone_extent", c_f32), ("split_n", c_i32), ("opacity_min", c_f32),
                ("radius_max", c_f32)]


class GsAttrs(ctypes.Structure):
    _fields_ = [("n_chan", c_i32), ("is_complex", c_i32), ("data", c_p), ("query_stride", c_i64)]


class GsQueries(ctypes.Structure):
    _fields_ = [("count", c_i32), ("rx", c_p), ("tx", c_p)]


class GsGrid(ctypes.Structure):
    _fields_ = [("H", c_i32), ("W", c_i32), ("tile_h", c_i32), ("tile_w", c_i32), ("view", ctypes.c_double * 9)]


class GsParams(ctypes.Structure):
    _fields_ = [("alpha_min", c_f32), ("alpha_max", c_f32), ("T_min", c_f32), ("dilation", c_f32),
                ("r_near", c_f32), ("atten_power", c_f32), ("atten_ref", c_i32), ("margin", c_f32),
                ("pair_capacity", c_i64), ("chan_group", c_i32), ("options", c_i32)]

GS_OPT_FORWARD_ONLY = 1
GS_OPT_BWD_PER_GROUP = 2
GS_OPT_BLEND_PER_GROUP = 4


class GsFlags(ctypes.Structure):
    _fields_ = [("n_visible", c_u32), ("n_pairs", c_u32), ("overflow", c_u32), ("n_invalid", c_u32)]


class GsMlp(ctypes.Structure):
    _fields_ = [("W1", c_p), ("b1", c_p), ("W2", c_p), ("b2", c_p), ("W3", c_p), ("b3", c_p),
                ("box_lo", c_f32 * 3), ("box_hi", c_f32 * 3), ("r_near", c_f32), ("n_chan", c_i32)]


class GsMlpRows(ctypes.Structure):
    _fields_ = [("n_sets", c_i32), ("tx", c_p), ("list", c_p), ("list_stride", c_i64), ("count", c_p),
                ("count_stride", c_i32), ("row_cap", c_i64), ("grid_x", c_i32)]


class GsMlpState(ctypes.Structure):
    _fields_ = [("cb", c_p), ("genc", c_p), ("save_h1", c_p), ("save_h2", c_p), ("save_do", c_p),
                ("save_dz2", c_p), ("save_dz1", c_p), ("dc", c_p), ("wT", c_p), ("partial", c_p),
                ("n_partial", c_i32)]


class GsMlpGrads(ctypes.Structure):
    _fields_ = [("dW1", c_p), ("db1", c_p), ("dW2", c_p), ("db2", c_p), ("dW3", c_p), ("db3", c_p), ("dE", c_p)]


class GsAdamSegment(ctypes.Structure):
    _fields_ = [("p", c_p), ("g", c_p), ("m", c_p), ("v", c_p), ("shadow", c_p), ("count", c_i64), ("lr", c_f32)]


class GsL2Grad(ctypes.Structure):
    _fields_ = [("partial", c_p), ("target", c_p), ("mean_grad", c_p), ("scale", c_f32)]


class GsTrainTarget(ctypes.Structure):
    _fields_ = [("target", c_p), ("target_mean", c_p), ("lambda_ch", c_f32), ("loss", c_p), ("h_hat", c_p),
                ("grad_scale", c_p)]


GS_BWD_ATTR_GRAD_ZEROED = 1
GS_TRAIN_WRITE_SPECTRUM = 2
GS_TRAIN_DEFER_GEOMETRY = 4
GS_TIMER_BLEND, GS_TIMER_BLEND_BWD, GS_TIMER_TRAIN = 0, 1, 2


class GsBatchJob(ctypes.Structure):
    _fields_ = [("scene", GsScene), ("attrs", GsAttrs), ("queries", GsQueries), ("grid", GsGrid),
                ("params", GsParams), ("spectrum", c_p), ("workspace", c_p), ("workspace_bytes", c_sz)]


class GsBatchInfo(ctypes.Structure):
    _fields_ = [("items", c_i64), ("n_queries", c_i32), ("block", c_i32), ("workgroups", c_i32),
                ("reserved", c_i32)]


_LAYOUT_FIELDS = ["total", "flags", "rec", "rect", "status", "tinfo", "order", "keys", "pair_keys", "pair_list",
                  "ranges", "T_final", "n_last", "n_contrib", "flags_stride", "rec_stride", "rect_stride",
                  "status_stride", "tinfo_stride", "order_stride", "keys_stride", "pair_keys_stride",
                  "pair_list_stride", "ranges_stride", "pix_stride"]


class GsLayout(ctypes.Structure):
    _fields_ = [(f, c_sz) for f in _LAYOUT_FIELDS] + [("pair_capacity", c_i64), ("tiles_x", c_i32),
                                                        ("tiles_y", c_i32)]


# every symbol declared in include/gsparc.h, with (restype, argtypes)
SIGNATURES = {
    "gs_default_params": (None, [ctypes.POINTER(GsParams)]),
    "gs_default_grid": (None, [ctypes.POINTER(GsGrid), c_i32, c_i32]),
    "gs_status_string": (ctypes.c_char_p, [c_i32]),
    "gs_workspace_layout": (c_i32, [c_i32, c_i32, ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams),
                                    ctypes.POINTER(GsLayout)]),
    "gs_render_forward": (c_i32, [ctypes.POINTER(GsScene), ctypes.POINTER(GsAttrs), ctypes.POINTER(GsQueries),
                                  ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams), c_p, c_p, c_sz, c_p]),
    "gs_render_prepare": (c_i32, [ctypes.POINTER(GsScene), ctypes.POINTER(GsQueries), ctypes.POINTER(GsGrid),
                                  ctypes.POINTER(GsParams), c_p, c_sz, c_p]),
    "gs_render_blend": (c_i32, [ctypes.POINTER(GsAttrs), c_i32, c_i32, c_i32, ctypes.POINTER(GsGrid),
                                ctypes.POINTER(GsParams), c_p, c_p, c_sz, c_p]),
    "gs_render_blend_loss": (c_i32, [ctypes.POINTER(GsAttrs), c_i32, c_i32, c_i32, ctypes.POINTER(GsGrid),
                                     ctypes.POINTER(GsParams), c_p, c_p, c_sz, c_p, c_f32, c_p, c_p, c_p, c_p, c_p,
                                     c_sz, c_p]),
    "gs_render_backward": (c_i32, [ctypes.POINTER(GsScene), ctypes.POINTER(GsAttrs), ctypes.POINTER(GsQueries),
                                   c_i32, ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams), c_p, c_p, c_p, c_p,
                                   c_p, c_p, c_p, c_i32, c_p, c_sz, c_p]),
    "gs_render_backward_l2": (c_i32, [ctypes.POINTER(GsScene), ctypes.POINTER(GsAttrs), ctypes.POINTER(GsQueries),
                                      c_i32, ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams), c_p,
                                      ctypes.POINTER(GsL2Grad), c_p, c_p, c_p, c_p, c_p, c_i32, c_p, c_sz, c_p]),
    "gs_loss_spectrum_stats": (c_i32, [c_p, c_p, c_i32, c_i32, c_i32, c_i32, c_i32, c_f32, c_p, c_p, c_p, c_p, c_p,
                                       c_sz, c_p]),
    "gs_loss_l1_ssim_scratch_bytes": (c_sz, [c_i32, c_i32, c_i32, c_i32]),
    "gs_loss_l1_ssim": (c_i32, [c_p, c_p, c_i32, c_i32, c_i32, c_i32, c_f32, c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "gs_spatial_mean": (c_i32, [c_p, c_i32, c_i32, c_i32, c_i32, c_i32, c_p, c_p]),
    "gs_train_scratch_bytes": (c_sz, [c_i32, c_i32, ctypes.POINTER(GsGrid)]),
    "gs_render_train": (c_i32, [ctypes.POINTER(GsScene), ctypes.POINTER(GsAttrs), ctypes.POINTER(GsQueries), c_i32,
                                ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams), c_p, c_p,
                                ctypes.POINTER(GsTrainTarget), c_p, c_p, c_p, c_p, c_p, c_p, c_i32, c_p, c_sz, c_p,
                                c_sz, c_p]),
    "gs_render_train_geometry": (c_i32, [ctypes.POINTER(GsScene), ctypes.POINTER(GsQueries), ctypes.POINTER(GsGrid),
                                         ctypes.POINTER(GsParams), c_p, c_p, c_p, c_p, c_p, c_sz, c_p]),
    "gs_render_live": (c_i32, [c_i32, c_i32, ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams), c_p, c_sz, c_p,
                               c_i64, c_p, c_p]),
    "gs_loss_spectrum": (c_i32, [c_p, c_p, c_i32, c_i32, c_i32, c_i32, c_i32, c_f32, c_p, c_p, c_p, c_p, c_sz,
                                 c_p]),
    "gs_loss_spectrum_noalloc": (c_i32, [c_p, c_p, c_i32, c_i32, c_i32, c_i32, c_i32, c_f32, c_p, c_p, c_p, c_p]),
    "gs_mlp_embed": (c_i32, [ctypes.POINTER(GsMlp), c_p, c_i32, c_p, c_p]),
    "gs_mlp_forward": (c_i32, [ctypes.POINTER(GsMlp), c_p, c_p, c_i32, ctypes.POINTER(GsMlpRows), c_p, c_i64,
                               ctypes.POINTER(GsMlpState), c_p]),
    "gs_mlp_backward": (c_i32, [ctypes.POINTER(GsMlp), c_p, c_p, c_i32, ctypes.POINTER(GsMlpRows), c_p, c_i64,
                                c_i32, ctypes.POINTER(GsMlpState), ctypes.POINTER(GsMlpGrads), c_p]),
    "gs_adam_step": (c_i32, [ctypes.POINTER(GsAdamSegment), c_i32, c_i32, c_f32, c_f32, c_f32, c_p, c_p, c_p]),
    "gs_adam_step_scheduled": (c_i32, [ctypes.POINTER(GsAdamSegment), ctypes.POINTER(c_f32), c_i32, c_i32, c_p,
                                       c_f32, c_f32, c_f32, c_p, c_p, c_p]),
    "gs_overflow_word": (c_i32, [c_p, c_sz, c_i32, c_i32, ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams), c_i32,
                                 ctypes.POINTER(c_p)]),
    "gs_emission_forward": (c_i32, [c_p, c_i64, c_i32, c_p, c_i32, c_p, c_p, c_i32, c_f32, c_p, c_i64, c_p]),
    "gs_emission_backward": (c_i32, [c_p, c_i64, c_i32, c_p, c_i32, c_p, c_p, c_i32, c_f32, c_p, c_i64, c_p, c_p,
                                     c_p]),
    "gs_confidence_scratch_bytes": (c_sz, [c_i32]),
    "gs_densify_stats": (c_i32, [c_p, c_i32, c_p, c_p, c_p, c_p, c_p]),
    "gs_densify_scratch_bytes": (c_sz, [c_i32]),
    "gs_densify_plan": (c_i32, [c_i32, c_p, c_p, c_p, c_p, c_p, ctypes.POINTER(GsDensifyParams), c_p, c_p, c_i64,
                                c_p, c_p, c_sz, c_p]),
    "gs_densify_apply": (c_i32, [c_i32, c_i32, c_p, c_p, ctypes.POINTER(GsScene), c_p, c_i32, c_p, c_p, c_p, c_p,
                                 c_p]),
    "gs_densify_gather": (c_i32, [c_i32, c_i32, c_p, c_p, c_p, c_p, c_i32, c_i32, c_i32, c_p]),
    "gs_opacity_reset": (c_i32, [c_i32, c_p, c_f32, c_p]),
    "gs_screen_radius": (c_i32, [c_p, c_sz, c_i32, c_i32, ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams), c_i32,
                                 c_p, c_p]),
    "gs_confidence_loss": (c_i32, [c_p, c_p, c_i32, c_p, c_p, c_p, c_p, c_f32, c_p, c_p, c_p, c_p, c_p, c_p, c_p,
                                   c_sz, c_p]),
    "gs_batch_plan_bytes": (c_sz, [c_i32]),
    "gs_batch_plan": (c_i32, [ctypes.POINTER(GsBatchJob), c_i32, c_p, c_sz, ctypes.POINTER(GsBatchInfo), c_p]),
    "gs_batch_run": (c_i32, [ctypes.POINTER(GsBatchJob), c_i32, c_p, c_sz, c_i32, c_p, c_p]),
    "gs_wall_clock_khz": (c_i32, [ctypes.POINTER(c_i32)]),
    "gs_timing_enable": (c_i32, [c_i32]),
    "gs_timing_read": (c_i32, [c_i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(c_i64)]),
    "gs_check": (c_i32, [c_p, c_sz, c_i32, c_i32, ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams), c_p]),
    "gs_read_flags": (c_i32, [c_p, c_sz, c_i32, c_i32, ctypes.POINTER(GsGrid), ctypes.POINTER(GsParams),
                              ctypes.POINTER(GsFlags), c_p]),
}

_lib = None


class GsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        msg = lib().gs_status_string(status).decode() if _lib is not None else str(status)
        super().__init__("%s: %s (status %d)" % (what, msg, status))


def lib():
    """Loads libgsparc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgsparc.so is not built (run python -m paper_2511_22793_amd.build); "
                               "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, what: str):
    if status != GS_OK:
        raise GsError(status, what)
