"""ctypes declarations mirroring ``include/emrt.h`` (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libemrt.so")

EMRT_OK = 0
EMRT_W_PATHS_TRUNCATED = 1
EMRT_W_CACHE_FULL = 2
EMRT_E_INVALID = -1
EMRT_E_STATE = -2
EMRT_E_WORKSPACE = -3
EMRT_E_HIP = -4
EMRT_E_UNSUPPORTED = -5
EMRT_E_DEVICE_FLAG = -6
STATIC_WORKSPACE_BYTES = 64 << 20  # EMRT_STATIC_WORKSPACE_BYTES
CAPTURE_LOG_ROWS = 1 << 16  # EMRT_CAPTURE_LOG_ROWS

c_i32, c_i64, c_u32, c_f64, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p


class Config(ctypes.Structure):
    _fields_ = [
        ("n_freq", c_i32), ("freq_hz", c_f64 * 4), ("max_reflections", c_i32), ("diffraction", c_i32),
        ("rays_per_tx", c_i32), ("rx_sphere_k", c_f64), ("diff_max_leg_m", c_f64), ("tx_power_w", c_f64),
        ("antenna_mode", c_i32), ("path_cap_per_link", c_i32), ("path_capacity", c_i64), ("table_capacity", c_i64),
        ("adjoint_materials", c_i32), ("dyn_rebuild_ratio", c_f64), ("ray_regroup", c_i32),
    ]


class Sizes(ctypes.Structure):
    _fields_ = [("n_verts", c_i64), ("n_tris", c_i64), ("n_faces", c_i64), ("n_objects", c_i64),
                ("n_tx", c_i32), ("n_rx", c_i32)]


class SceneDesc(ctypes.Structure):
    _fields_ = [("n_verts", c_i64), ("n_tris", c_i64), ("n_faces", c_i64), ("n_objects", c_i64),
                ("verts", c_vp), ("tris", c_vp), ("tri_face", c_vp), ("face_object", c_vp), ("face_material", c_vp),
                ("object_dynamic", c_vp), ("n_materials", c_i32), ("material_eps", c_vp)]


class FrameDesc(ctypes.Structure):
    _fields_ = [("frame", c_i64), ("t_s", c_f64), ("n_tx", c_i32), ("n_rx", c_i32), ("obj_xform", c_vp),
                ("obj_vel", c_vp), ("tx_pos", c_vp), ("tx_vel", c_vp), ("tx_orient", c_vp), ("rx_pos", c_vp),
                ("rx_vel", c_vp)]


class ChannelView(ctypes.Structure):
    _fields_ = [("H", c_vp), ("P_coh", c_vp), ("P_inc", c_vp), ("tau_mean", c_vp), ("tau_rms", c_vp),
                ("fd_mean", c_vp), ("fd_rms", c_vp), ("n_paths", c_vp), ("flags", c_vp)]


class PathView(ctypes.Structure):
    _fields_ = [("cap", c_i32), ("key", c_vp), ("tri_ids", c_vp), ("a", c_vp), ("tau", c_vp), ("fd", c_vp),
                ("angles", c_vp), ("count", c_vp)]


CORR_LAGS = 4


class CoherenceView(ctypes.Structure):
    _fields_ = [("tc", c_vp), ("corr", c_vp), ("trigger", c_vp)]


class Stats(ctypes.Structure):
    _fields_ = [("rays_per_bounce", c_i64 * 7), ("n_candidates", c_i64), ("n_valid", c_i64), ("n_cache", c_i64),
                ("node_visits", c_i64), ("tri_tests", c_i64), ("segments", c_i64), ("captures", c_i64),
                ("n_static_tris", c_i64), ("n_dynamic_tris", c_i64), ("n_edges", c_i64), ("device_flags", c_u32),
                ("bounce_ms", c_f64), ("bounce_launches", c_i32), ("validate_ms", c_f64),
                ("validate_launches", c_i32), ("static_tree_area", c_f64), ("wide_box_tests", c_i64),
                ("dyn_rebuilds", c_i64), ("dyn_tree_quality", c_f64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "emrt_config_default": (None, [ctypes.POINTER(Config)]),
    "emrt_ctx_create": (c_i32, [ctypes.POINTER(Config), ctypes.POINTER(c_vp)]),
    "emrt_ctx_destroy": (c_i32, [c_vp]),
    "emrt_workspace_size": (c_i32, [c_vp, ctypes.POINTER(Sizes), ctypes.POINTER(ctypes.c_size_t)]),
    "emrt_bind_workspace": (c_i32, [c_vp, c_vp, ctypes.c_size_t]),
    "emrt_bind_static_workspace": (c_i32, [c_vp]),
    "emrt_set_stream": (c_i32, [c_vp, c_vp]),
    "emrt_set_scene": (c_i32, [c_vp, ctypes.POINTER(SceneDesc)]),
    "emrt_set_materials": (c_i32, [c_vp, c_vp, c_i32]),
    "emrt_set_reflection_coefficients": (c_i32, [c_vp, c_vp, c_i32]),
    "emrt_set_frame": (c_i32, [c_vp, ctypes.POINTER(FrameDesc)]),
    "emrt_set_frame_host": (c_i32, [c_vp, ctypes.POINTER(FrameDesc)]),
    "emrt_step": (c_i32, [c_vp, c_i32]),
    "emrt_step_rx": (c_i32, [c_vp, c_vp, c_i32, c_i32]),
    "emrt_read_channels": (c_i32, [c_vp, ctypes.POINTER(ChannelView)]),
    "emrt_read_paths": (c_i32, [c_vp, ctypes.POINTER(PathView)]),
    "emrt_backward": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "emrt_read_coherence": (c_i32, [c_vp, c_f64, ctypes.POINTER(CoherenceView), ctypes.POINTER(c_f64),
                                    ctypes.POINTER(c_i64)]),
    "emrt_coherence_reset": (c_i32, [c_vp]),
    "emrt_batch_create": (c_i32, [ctypes.POINTER(c_vp), c_i32, ctypes.POINTER(c_vp)]),
    "emrt_batch_destroy": (c_i32, [c_vp]),
    "emrt_batch_workspace_size": (c_i32, [c_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "emrt_batch_bind_workspace": (c_i32, [c_vp, c_vp, ctypes.c_size_t]),
    "emrt_batch_set_stream": (c_i32, [c_vp, c_vp]),
    "emrt_batch_set_options": (c_i32, [c_vp, c_i32, c_i32, c_i32, c_i32]),
    "emrt_batch_step": (c_i32, [c_vp, c_i32]),
    "emrt_batch_autotune": (c_i32, [c_vp, c_i32, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                                    ctypes.POINTER(c_i32)]),
    "emrt_batch_sync": (c_i32, [c_vp]),
    "emrt_batch_last_error": (c_i32, [c_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "emrt_debug_ray_records": (c_i32, [c_vp, c_i32, c_vp, c_i32, c_vp]),
    "emrt_debug_select_rays": (c_i32, [c_vp, c_i32, c_vp, c_i32]),
    "emrt_debug_ray_captures": (c_i32, [c_vp, c_vp, c_i64, c_vp]),
    "emrt_cache_size": (c_i32, [c_vp, ctypes.POINTER(c_i64)]),
    "emrt_cache_export": (c_i32, [c_vp, c_vp, c_i64, ctypes.POINTER(c_i64)]),
    "emrt_cache_import": (c_i32, [c_vp, c_vp, c_i64]),
    "emrt_read_stats": (c_i32, [c_vp, ctypes.POINTER(Stats)]),
    "emrt_set_instrumentation": (c_i32, [c_vp, c_i32, c_i32]),
    "emrt_sync": (c_i32, [c_vp]),
    "emrt_status_string": (ctypes.c_char_p, [c_i32]),
    "emrt_last_error": (c_i32, [c_vp, ctypes.c_char_p, ctypes.c_size_t]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libemrt.so not found at {path}: build it with __graft_entry__.build() "
                           "or python paper_2303_10521_amd/build.py")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
