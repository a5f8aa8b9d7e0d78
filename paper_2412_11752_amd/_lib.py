"""ctypes declarations of libdrk's C ABI (include/drk.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdrk.so")

DRK_OK, DRK_EINVAL, DRK_ENOMEM, DRK_EOVERFLOW, DRK_EAGAIN, DRK_ENOTFOUND, DRK_EDEVICE = range(7)
STATUS_NAMES = {0: "DRK_OK", 1: "DRK_EINVAL", 2: "DRK_ENOMEM", 3: "DRK_EOVERFLOW", 4: "DRK_EAGAIN",
                5: "DRK_ENOTFOUND", 6: "DRK_EDEVICE"}

EXPORTED = [
    "drk_opts_default", "drk_last_error", "drk_version", "drk_ws_create", "drk_ws_destroy", "drk_ws_size_query",
    "drk_preprocess", "drk_bin_sort", "drk_render_fwd", "drk_render_trace", "drk_trace_metrics",
    "drk_render_depth_normal", "drk_mesh_to_drk", "drk_activate", "drk_activate_bwd", "drk_adam_step",
    "drk_render_bwd",
    "drk_render_fwd_noalloc", "drk_ws_generation", "drk_ws_status", "drk_ws_export",
    "drk_serve_create", "drk_serve_destroy", "drk_serve_add_scene", "drk_serve_submit", "drk_serve_poll",
]


class Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("K", C.c_int32), ("color_mode", C.c_int32), ("sh_degree", C.c_int32),
                ("reserved", C.c_int32), ("mu", C.c_void_p), ("q", C.c_void_p), ("scale", C.c_void_p),
                ("theta", C.c_void_p), ("eta", C.c_void_p), ("tau", C.c_void_p), ("opacity", C.c_void_p),
                ("color", C.c_void_p)]


class SceneGrad(C.Structure):
    _fields_ = [("mu", C.c_void_p), ("q", C.c_void_p), ("scale", C.c_void_p), ("theta", C.c_void_p),
                ("eta", C.c_void_p), ("tau", C.c_void_p), ("opacity", C.c_void_p), ("color", C.c_void_p)]


class SceneOut(C.Structure):
    _fields_ = SceneGrad._fields_


class Camera(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float), ("R", C.c_float * 9), ("t", C.c_float * 3),
                ("bg", C.c_float * 3)]


class Opts(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("alpha_max", C.c_float), ("T_min", C.c_float),
                ("near_plane", C.c_float), ("lowpass_sl", C.c_float), ("cache_len", C.c_int32),
                ("cull_mode", C.c_int32), ("validate", C.c_int32), ("key_mode", C.c_int32),
                ("launch_order", C.c_int32), ("counters", C.c_int32)]


class ServeCfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_inflight", C.c_int32), ("queue_capacity", C.c_int32),
                ("use_graphs", C.c_int32), ("initial_pairs", C.c_int32), ("opts", Opts)]


class ReqStats(C.Structure):
    _fields_ = [("submit_us", C.c_double), ("start_us", C.c_double), ("done_us", C.c_double),
                ("pairs", C.c_int64), ("status", C.c_int32), ("width", C.c_int32), ("height", C.c_int32)]


class DrkError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib() -> C.CDLL:
    """Load libdrk.so from the package directory.  Raises if it has not been built: there is no
    fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2412_11752_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    L.drk_opts_default.restype = Opts
    L.drk_last_error.restype = C.c_char_p
    L.drk_version.restype = C.c_char_p
    sig = {
        "drk_ws_create": [i64, i32, i32, i32, i32, i64, C.POINTER(vp)],
        "drk_ws_destroy": [vp],
        "drk_ws_size_query": [i64, i32, i32, i32, i32, i64, C.POINTER(C.c_size_t)],
        "drk_preprocess": [vp, C.POINTER(Scene), C.POINTER(Camera), i32, C.POINTER(Opts), vp],
        "drk_bin_sort": [vp, vp],
        "drk_render_fwd": [vp, vp, vp, vp],
        "drk_render_trace": [vp, vp, vp, i32, vp, vp, vp, vp],
        "drk_trace_metrics": [vp, vp, i64, i32, vp, vp],
        "drk_render_depth_normal": [vp, vp, vp, vp, vp, vp],
        "drk_mesh_to_drk": [vp, i64, vp, i64, i32, vp, i32, C.c_float, C.c_float, C.POINTER(SceneOut), vp, vp],
        "drk_activate": [C.POINTER(Scene), C.POINTER(SceneOut), vp],
        "drk_activate_bwd": [C.POINTER(Scene), C.POINTER(SceneGrad), C.POINTER(SceneOut), vp],
        "drk_adam_step": [vp, vp, vp, vp, i64, C.c_float, C.c_float, C.c_float, C.c_float, i32, vp],
        "drk_render_bwd": [vp, C.POINTER(Scene), vp, vp, C.POINTER(SceneGrad), vp],
        "drk_render_fwd_noalloc": [C.POINTER(Scene), C.POINTER(Camera), C.POINTER(Opts), vp, vp, vp],
        "drk_ws_generation": [vp, C.POINTER(C.c_uint64)],
        "drk_ws_status": [vp, vp, C.POINTER(i64)],
        "drk_ws_export": [vp, i32, i32, vp, i64, C.POINTER(i64), vp],
        "drk_serve_create": [C.POINTER(ServeCfg), C.POINTER(vp)],
        "drk_serve_destroy": [vp],
        "drk_serve_add_scene": [vp, C.POINTER(Scene), C.POINTER(i32)],
        "drk_serve_submit": [vp, i32, C.POINTER(Camera), vp, C.POINTER(C.c_uint64)],
        "drk_serve_poll": [vp, C.c_uint64, i32, C.POINTER(ReqStats)],
    }
    for name, args in sig.items():
        if not hasattr(L, name):
            continue
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int
    _lib = L
    return L


def check(code: int, what: str = "") -> None:
    if code != DRK_OK:
        msg = lib().drk_last_error().decode()
        raise DrkError(code, f"{what}: {msg}" if what else msg)
