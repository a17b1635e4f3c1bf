"""ctypes declarations of the C ABI in include/pfn.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpfn.so")

PFN_OK, PFN_ERR_INVALID_ARG, PFN_ERR_OUT_OF_MEMORY, PFN_ERR_HIP = 0, -1, -2, -3
PFN_ERR_NOT_READY, PFN_ERR_UNSUPPORTED, PFN_ERR_NUMERIC = -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "OUT_OF_MEMORY", -3: "HIP", -4: "NOT_READY",
                -5: "UNSUPPORTED", -6: "NUMERIC"}
PFN_F32, PFN_F16, PFN_BF16 = 0, 1, 2
INDIRECT_NONE, INDIRECT_CACHE, INDIRECT_FIELD = 0, 1, 2
DIRECT_SHADOW_RAYS, DIRECT_LIGHT_VOLUME = 0, 1
TK_MARCH, TK_TRACE, TK_TRAIN, TK_PT, TK_QUERY, TK_ADAM = 0, 1, 2, 3, 4, 5
TK_WF_MARCH, TK_WF_ENCODE, TK_WF_FIELD, TK_WF_RESOLVE = 6, 7, 8, 9
TK_FI_SAMPLE, TK_FI_NEE, TK_PM_ESTIMATE, TK_WF_DIR = 10, 11, 12, 13


class PointLight(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("intensity", C.c_float * 3)]


class TraceParams(C.Structure):
    _fields_ = [("n_photons", C.c_uint64), ("n_bins", C.c_int), ("g_bins", C.c_float * 8),
                ("cache_res", C.c_int), ("max_collisions", C.c_int), ("rr_start", C.c_int),
                ("seed", C.c_uint64)]


class TraceStats(C.Structure):
    _fields_ = [("n_records", C.c_uint64), ("n_records_dropped", C.c_uint64),
                ("emitted", C.c_double * 3), ("entered", C.c_double * 3),
                ("escaped", C.c_double * 3), ("escaped_uncollided", C.c_double * 3),
                ("absorbed", C.c_double * 3), ("truncated", C.c_double * 3),
                ("rr_killed", C.c_double * 3), ("stored", C.c_double * 3),
                ("collisions", C.c_double), ("null_events", C.c_double), ("kappa", C.c_double)]


class FieldDesc(C.Structure):
    _fields_ = [("levels", C.c_int), ("feats_per_level", C.c_int), ("base_res", C.c_int),
                ("growth", C.c_float), ("log2_table", C.c_int), ("hidden_layers", C.c_int),
                ("width", C.c_int), ("psi", C.c_float)]


class TrainParams(C.Structure):
    _fields_ = [("steps", C.c_int), ("log2_batch", C.c_int), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("decay", C.c_float), ("decay_start", C.c_int), ("decay_interval", C.c_int),
                ("precision", C.c_int), ("seed", C.c_uint64), ("target", C.c_int),
                ("knn_k", C.c_int), ("radius", C.c_float), ("staggered", C.c_int),
                ("loss", C.c_int), ("g_sampling", C.c_int)]


class CameraS(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("target", C.c_float * 3), ("up", C.c_float * 3),
                ("fov_y_deg", C.c_float), ("width", C.c_int), ("height", C.c_int)]


class RenderParams(C.Structure):
    _fields_ = [("spp", C.c_int), ("step_voxels", C.c_float), ("max_steps", C.c_int),
                ("t_min", C.c_float), ("field_stride", C.c_int), ("g", C.c_float),
                ("indirect", C.c_int), ("direct", C.c_int), ("field_precision", C.c_int),
                ("light_mask", C.c_int), ("field_slot", C.c_int), ("seed", C.c_uint64)]


class RenderJob(C.Structure):
    _fields_ = [("cam", CameraS), ("params", RenderParams), ("dev_rgb_out", C.c_void_p)]


vp = C.c_void_p
ctxp = C.c_void_p
SIGNATURES = {
    "pfn_create": (C.c_int, [C.c_int, vp, C.POINTER(ctxp)]),
    "pfn_destroy": (None, [ctxp]),
    "pfn_last_error": (C.c_char_p, [ctxp]),
    "pfn_sync": (C.c_int, [ctxp]),
    "pfn_set_stream": (C.c_int, [ctxp, vp]),
    "pfn_set_volume": (C.c_int, [ctxp, vp, C.c_int, C.c_int, C.c_int, C.c_int]),
    "pfn_set_transfer_function": (C.c_int, [ctxp, C.POINTER(C.c_float), C.c_float]),
    "pfn_set_lights": (C.c_int, [ctxp, C.POINTER(PointLight), C.c_int]),
    "pfn_build_light_volume": (C.c_int, [ctxp, C.c_float]),
    "pfn_get_light_volume": (C.c_int, [ctxp, vp, C.c_size_t]),
    "pfn_trace_photon_cache": (C.c_int, [ctxp, C.POINTER(TraceParams), C.POINTER(TraceStats)]),
    "pfn_get_records": (C.c_int, [ctxp, vp, vp, vp, vp, vp, C.c_uint64, C.POINTER(C.c_uint64)]),
    "pfn_get_cache": (C.c_int, [ctxp, vp, C.c_size_t]),
    "pfn_set_cache": (C.c_int, [ctxp, vp, C.c_int, C.POINTER(C.c_float), C.c_int, C.c_double]),
    "pfn_cache_info": (C.c_int, [ctxp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                 C.POINTER(C.c_double)]),
    "pfn_field_select": (C.c_int, [ctxp, C.c_int]),
    "pfn_field_init": (C.c_int, [ctxp, C.POINTER(FieldDesc), C.c_uint64]),
    "pfn_field_num_params": (C.c_int, [ctxp, C.POINTER(C.c_size_t)]),
    "pfn_field_get_params": (C.c_int, [ctxp, vp, C.c_size_t]),
    "pfn_field_set_params": (C.c_int, [ctxp, vp, C.c_size_t]),
    "pfn_field_set_kappa": (C.c_int, [ctxp, C.c_double]),
    "pfn_field_query": (C.c_int, [ctxp, C.c_int, vp, vp, vp, C.c_int64, vp, vp]),
    "pfn_field_forward_backward": (C.c_int, [ctxp, C.c_int, vp, vp, vp, vp, C.c_int64, C.c_int,
                                             C.POINTER(C.c_double), vp]),
    "pfn_train_field": (C.c_int, [ctxp, C.POINTER(TrainParams), C.POINTER(C.c_float)]),
    "pfn_train_batch": (C.c_int, [ctxp, C.c_uint64, C.c_int64, C.c_int64, C.c_int, vp, vp, vp,
                                  vp, vp]),
    "pfn_field_adam_step": (C.c_int, [ctxp, vp, C.c_int64, C.c_float, C.c_float, C.c_float,
                                      C.c_float]),
    "pfn_render_frame": (C.c_int, [ctxp, C.POINTER(CameraS), C.POINTER(RenderParams), vp]),
    "pfn_render_first_interaction": (C.c_int, [ctxp, C.POINTER(CameraS), C.POINTER(RenderParams),
                                               vp]),
    "pfn_photon_map_build": (C.c_int, [ctxp, C.c_int]),
    "pfn_train_step_radius": (C.c_int, [C.POINTER(TrainParams), C.c_int, C.POINTER(C.c_float)]),
    "pfn_train_lr_at": (C.c_int, [C.POINTER(TrainParams), C.c_int, C.POINTER(C.c_float)]),
    "pfn_photon_map_set": (C.c_int, [ctxp, vp, vp, vp, vp, C.c_uint64, C.c_int,
                                     C.POINTER(C.c_float), C.c_int]),
    "pfn_photon_map_get": (C.c_int, [ctxp, vp, C.c_size_t, vp, vp, vp, C.c_uint64,
                                     C.POINTER(C.c_uint64)]),
    "pfn_photon_map_estimate": (C.c_int, [ctxp, vp, vp, vp, C.c_int64, C.c_float, C.c_int, vp,
                                          vp, vp]),
    "pfn_render_batch": (C.c_int, [ctxp, C.POINTER(RenderJob), C.c_int]),
    "pfn_render_path_traced": (C.c_int, [ctxp, C.POINTER(CameraS), C.c_int, C.c_int, C.c_float,
                                         C.c_int, C.c_int, C.c_uint64, vp]),
    "pfn_image_error": (C.c_int, [ctxp, vp, vp, C.c_int64, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "pfn_image_error_noalloc": (C.c_int, [ctxp, vp, vp, C.c_int64, vp]),
    "pfn_set_tile_config": (C.c_int, [ctxp, C.c_int, C.c_int, C.c_int]),
    "pfn_set_launch_mode": (C.c_int, [ctxp, C.c_int, C.c_int]),
    "pfn_set_render_strategy": (C.c_int, [ctxp, C.c_int]),
    "pfn_autotune_batch": (C.c_int, [ctxp, C.POINTER(RenderJob), C.c_int, C.c_int,
                                     C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int), C.POINTER(C.c_int),
                                     C.POINTER(C.c_double)]),
    "pfn_timing_enable": (C.c_int, [ctxp, C.c_int]),
    "pfn_timing_get": (C.c_int, [ctxp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "pfn_timing_reset": (C.c_int, [ctxp]),
    "pfn_count_enable": (C.c_int, [ctxp, C.c_int]),
    "pfn_count_get": (C.c_int, [ctxp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
}

_lib = None


class LibraryMissing(RuntimeError):
    pass


def load():
    """Load the in-tree HIP library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
