"""ctypes binding of libgsmi.so (the C ABI declared in include/gs.h).

Argument marshalling only: every step of the training path runs in the HIP
kernels of the library.  Loading fails loudly when the library is missing;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GSMI_LIB", os.path.join(_HERE, "libgsmi.so"))

GS_OK, GS_ERR_ARG, GS_ERR_HIP, GS_ERR_CAPACITY, GS_ERR_NONFINITE, GS_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
GS_MAX_SLOTS = 1024
GS_REC_STRIDE = 12
GS_DREC_STRIDE = 9
GS_STATUS_WORDS = 4
GS_FLAG_CAPACITY = 1
GS_FLAG_NONFINITE = 2
GS_BWD_STORED, GS_BWD_RECOMPUTE = 0, 1
GS_MAX_ADAM_GROUPS = 8

vp = C.c_void_p
i32, i64, f32, sz = C.c_int32, C.c_int64, C.c_float, C.c_size_t


class gs_gaussians(C.Structure):
    _fields_ = [("mean", vp), ("log_scale", vp), ("quat", vp), ("opacity_logit", vp),
                ("color", vp), ("n", i64), ("sh_degree", i32), ("reserved", i32)]


class gs_grads(C.Structure):
    _fields_ = [("mean", vp), ("log_scale", vp), ("quat", vp), ("opacity_logit", vp),
                ("color", vp), ("n", i64)]


class gs_views(C.Structure):
    _fields_ = [("n_slots", i32), ("total_pairs", i64), ("pair_offset", vp),
                ("gauss_offset", vp), ("cams", vp)]


class gs_tiling(C.Structure):
    _fields_ = [("width", i32), ("height", i32), ("tile_w", i32), ("tile_h", i32)]


class gs_projected(C.Structure):
    _fields_ = [("rec", vp), ("tile_bbox", vp), ("n_tiles", vp), ("m", i64)]


class gs_raster_plan(C.Structure):
    _fields_ = [("tile_order", vp), ("queue", vp), ("persistent_waves", i32), ("chunk", i32),
                ("chunk_offset", vp), ("chunk_items", vp), ("checkpoints", vp),
                ("max_items", i64), ("fwd_waves", i32), ("fwd_split", i32),
                ("dup_grads", vp), ("pair_first", vp), ("dup_capacity", i64),
                ("emit_idx", vp), ("chunk_last", vp)]


class gs_adam_group(C.Structure):
    _fields_ = [("param", vp), ("grad", vp), ("m", vp), ("v", vp), ("count", i64), ("lr", f32)]


class gs_mlp(C.Structure):
    _fields_ = [("w1", vp), ("w2", vp), ("w3", vp), ("b1", vp), ("b2", vp), ("b3", vp)]


class gs_mlp_grads(C.Structure):
    _fields_ = [("dw1", vp), ("dw2", vp), ("dw3", vp), ("db1", vp), ("db2", vp), ("db3", vp),
                ("dx", vp)]


class gs_gaussian_state(C.Structure):
    _fields_ = [("param", vp * 5), ("m", vp * 5), ("v", vp * 5), ("n", i64),
                ("color_rows", i32), ("reserved", i32)]


P = C.POINTER
F3 = f32 * 3

# name -> (restype, argtypes); every function the header declares
SIGNATURES = {
    "gs_project": (i32, [P(gs_gaussians), P(gs_views), P(gs_tiling), P(gs_projected), vp]),
    "gs_bin_sort_workspace_bytes": (sz, [i64, i64, P(gs_tiling), i32]),
    "gs_bin_sort": (i32, [P(gs_projected), P(gs_views), P(gs_tiling), i64, vp, sz, vp, vp, vp,
                          vp, vp, vp, vp]),
    "gs_raster_fwd": (i32, [P(gs_projected), P(gs_views), P(gs_tiling), vp, vp, P(f32), vp, vp,
                            vp, P(gs_raster_plan), vp]),
    "gs_raster_bwd": (i32, [P(gs_projected), P(gs_views), P(gs_tiling), vp, vp, P(f32), vp, vp,
                            vp, i32, vp, P(gs_raster_plan), vp]),
    "gs_raster_count": (i32, [P(gs_projected), P(gs_views), P(gs_tiling), vp, vp, vp, vp]),
    "gs_tile_order_workspace_bytes": (sz, [i64]),
    "gs_chunk_max_items": (i64, [i64, i64, i32]),
    "gs_chunk_items": (i32, [vp, i64, i32, i64, vp, vp, vp]),
    "gs_tile_order": (i32, [vp, i64, vp, sz, vp, vp]),
    "gs_project_bwd": (i32, [P(gs_gaussians), P(gs_views), P(gs_tiling), P(gs_projected), vp,
                             P(gs_grads), vp]),
    "gs_loss_workspace_bytes": (sz, [i32, i32, i32]),
    "gs_loss": (i32, [vp, vp, vp, i32, i32, i32, f32, f32, vp, sz, vp, vp, vp, vp]),
    "gs_loss_noalloc": (i32, [vp, vp, vp, i32, i32, i32, f32, f32, vp, vp, vp, vp]),
    "gs_graph_begin": (i32, [vp]),
    "gs_graph_end": (i32, [vp, P(vp)]),
    "gs_graph_launch": (i32, [vp, vp]),
    "gs_graph_destroy": (None, [vp]),
    "gs_adam": (i32, [P(gs_adam_group), i32, f32, f32, f32, i32, i32, vp]),
    "gs_adam_dev": (i32, [P(gs_adam_group), i32, P(f32), i32, f32, f32, f32, vp, i32, vp]),
    "gs_project_bwd_adam": (i32, [P(gs_gaussians), P(gs_views), P(gs_tiling), P(gs_projected),
                                  vp, P(gs_adam_group), i32, P(f32), i32, f32, f32, f32, i32, vp,
                                  vp]),
    "gs_peak_copy": (i32, [vp, vp, i64, vp]),
    "gs_peak_fma": (i32, [vp, i32, i32, vp]),
    "gs_peak_exp": (i32, [vp, i32, i32, vp]),
    "gs_peak_lds": (i32, [vp, i32, i32, vp]),
    "gs_peak_atomic": (i32, [vp, i64, i32, i32, i32, vp]),
    "gs_peak_mfma": (i32, [vp, i32, i32, vp]),
    "gs_densify_stats": (i32, [P(gs_views), P(gs_tiling), P(gs_projected), vp, i64, vp, vp, vp]),
    "gs_densify_workspace_bytes": (sz, [i64]),
    "gs_densify_select": (i32, [P(gs_gaussian_state), vp, vp, f32, f32, f32, f32, f32, vp, sz,
                                vp, vp, vp]),
    "gs_densify_apply": (i32, [P(gs_gaussian_state), vp, vp, vp, f32, P(gs_gaussian_state), vp]),
    "gs_opacity_reset": (i32, [P(gs_gaussian_state), f32, vp]),
    "gs_zero": (i32, [vp, sz, vp]),
    "gs_check_status": (i32, [vp, vp, P(i64)]),
    "gs_last_error": (C.c_char_p, []),
    "gs_version": (C.c_char_p, []),
    "gs_knn_workspace_bytes": (sz, [i64, i32]),
    "gs_knn": (i32, [vp, i64, i32, vp, sz, vp, vp, vp, vp]),
    "gs_plain_init_workspace_bytes": (sz, [i64]),
    "gs_plain_init": (i32, [vp, vp, i64, f32, vp, sz, vp, vp, vp, vp, vp, vp]),
    "gs_psnr_workspace_bytes": (sz, [i32, i32, i32]),
    "gs_masked_psnr": (i32, [vp, vp, vp, i32, i32, i32, vp, sz, vp, vp]),
    "gs_scale_rows": (i32, [vp, vp, i64, i64, vp]),
    "gs_mlp_features": (i32, [vp, vp, i64, vp, vp, vp, vp, vp]),
    "gs_mlp_fwd": (i32, [vp, i64, P(gs_mlp), vp, vp]),
    "gs_mlp_bwd_workspace_bytes": (sz, [i64]),
    "gs_mlp_bwd": (i32, [vp, i64, P(gs_mlp), vp, P(gs_mlp_grads), vp, sz, vp]),
    "gs_mlp_targets": (i32, [vp, vp, vp, vp, vp, i64, vp, vp]),
    "gs_mlp_loss_workspace_bytes": (sz, [i64]),
    "gs_mlp_loss": (i32, [vp, vp, i64, vp, vp, sz, vp, vp]),
    "gs_mlp_apply": (i32, [vp, vp, vp, i64, vp, vp, vp, vp]),
}

_lock = threading.Lock()
_lib = None


class GSError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


def load():
    """Load libgsmi.so; raises if it is missing (no fallback exists)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2509_12138_amd.build` "
                "(there is no fallback implementation)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            if not hasattr(lib, name):
                continue
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def exported_symbols():
    """Names from SIGNATURES that the loaded library exports."""
    lib = load()
    return [n for n in SIGNATURES if hasattr(lib, n)]


def last_error() -> str:
    return load().gs_last_error().decode()


def check(name, status):
    if status != GS_OK:
        raise GSError(name, status, last_error())
    return status


def call(name, *args):
    """Call a status-returning entry point and raise GSError on failure."""
    return check(name, getattr(load(), name)(*args))
