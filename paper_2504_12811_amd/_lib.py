"""ctypes binding of the C ABI in include/aaa.h (argument marshalling only).

Every step of the rendering path runs in the HIP library; this module only
converts Python objects to the ABI structs and raises on error codes.  It
fails loudly when the built library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaaa_hip.so")

AAA_OK, AAA_ERR_INVALID, AAA_ERR_WORKSPACE, AAA_ERR_PAIR_OVERFLOW, AAA_ERR_HIP, AAA_ERR_UNSUPPORTED = range(6)
AAA_FILTER_OFF, AAA_FILTER_VOLUME, AAA_NO_TILE_CULL, AAA_STATS, AAA_TIMING, AAA_LONG_ALL = 1, 2, 4, 8, 16, 32
AAA_WIDE_RANKS = 64
AAA_SUBTILE_SORT = 128
AAA_MAX_TRAIN_CAMERAS = 4096
AAA_STATIC_SLOT_BYTES = 64 << 20
STAGES = ["preprocess", "count", "scan", "write", "sort", "ranges", "blend", "frame"]

# Every symbol include/aaa.h declares (checked by the ABI test).
EXPORTS = [
    "aaa_create", "aaa_destroy", "aaa_last_error", "aaa_version", "aaa_workspace_size", "aaa_render",
    "aaa_stage_times", "aaa_workspace_size_batch", "aaa_render_batch", "aaa_render_backward_batch",
    "aaa_backward_scratch_size", "aaa_training_frequency", "aaa_adam_step",
    "aaa_render_backward", "aaa_render_backward_noalloc", "aaa_read_gaussians", "aaa_read_pairs",
    "aaa_sort_tmp_size", "aaa_sort_pairs", "aaa_measure_peaks",
]


class AAAError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"aaa error {code}: {msg}")
        self.code = code


class Scene(C.Structure):
    _fields_ = [("n", C.c_int64), ("sh_degree", C.c_int32), ("_pad", C.c_int32),
                ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p), ("v_train", C.c_void_p)]


class SceneGrad(C.Structure):
    _fields_ = [("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class Camera(C.Structure):
    _fields_ = [("viewmat", C.c_double * 16), ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double),
                ("cy", C.c_double), ("width", C.c_int32), ("height", C.c_int32), ("znear", C.c_double),
                ("bg", C.c_double * 3)]


class Settings(C.Structure):
    _fields_ = [("filter_k", C.c_double), ("ray_window", C.c_int32), ("flags", C.c_uint32),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double), ("t_min", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("pairs", C.c_uint64), ("visible", C.c_uint64), ("evaluations", C.c_uint64),
                ("contributors", C.c_uint64), ("candidate_tiles", C.c_uint64), ("near", C.c_uint64),
                ("wave_steps", C.c_uint64), ("wave_near_steps", C.c_uint64), ("wave_contrib_steps", C.c_uint64)]


_lib = None


def lib():
    """Load libaaa_hip.so (built in-tree by build.py); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2504_12811_amd.build` "
                               "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, i32, u64, i64 = C.c_void_p, C.c_int32, C.c_uint64, C.c_int64
        L.aaa_create.argtypes = [C.POINTER(vp), C.c_int]
        L.aaa_destroy.argtypes = [vp]
        L.aaa_destroy.restype = None
        L.aaa_last_error.restype = C.c_char_p
        L.aaa_version.restype = C.c_char_p
        L.aaa_workspace_size.argtypes = [C.POINTER(Scene), C.POINTER(Camera), C.POINTER(Settings), u64,
                                         C.POINTER(C.c_size_t)]
        L.aaa_render.argtypes = [vp, C.POINTER(Scene), C.POINTER(Camera), C.POINTER(Settings), vp, C.c_size_t, u64,
                                 vp, vp, vp, C.POINTER(Stats)]
        L.aaa_render_backward.argtypes = [vp, C.POINTER(Scene), C.POINTER(Camera), C.POINTER(Settings), vp, C.c_size_t,
                                          u64, vp, vp, vp, vp, C.c_size_t, C.POINTER(SceneGrad)]
        L.aaa_render_backward_noalloc.argtypes = [vp, C.POINTER(Scene), C.POINTER(Camera), C.POINTER(Settings), vp,
                                                  C.c_size_t, u64, vp, vp, vp, C.POINTER(SceneGrad)]
        L.aaa_adam_step.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int64, C.c_double, C.c_double, C.c_double,
                                    C.c_double, vp]
        L.aaa_training_frequency.argtypes = [vp, vp, C.c_int64, C.POINTER(Camera), C.c_int, vp, vp]
        L.aaa_backward_scratch_size.argtypes = [vp, C.POINTER(Scene), C.c_int, C.POINTER(Camera), C.POINTER(Settings),
                                                vp, C.c_size_t, u64, vp, C.POINTER(C.c_size_t)]
        L.aaa_read_gaussians.argtypes = [C.POINTER(Scene), C.POINTER(Camera), u64, vp, C.c_size_t, vp, vp, vp, vp, vp,
                                         vp]
        L.aaa_read_pairs.argtypes = [C.POINTER(Scene), C.POINTER(Camera), u64, vp, C.c_size_t, vp, vp, vp, vp, u64,
                                     C.POINTER(C.c_uint64)]
        L.aaa_workspace_size_batch.argtypes = [C.POINTER(Scene), C.c_int, C.POINTER(Camera), C.POINTER(Settings), u64,
                                               C.POINTER(C.c_size_t)]
        L.aaa_render_batch.argtypes = [vp, C.POINTER(Scene), C.c_int, C.POINTER(Camera), C.POINTER(Settings), vp,
                                       C.c_size_t, u64, vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(Stats)]
        L.aaa_render_backward_batch.argtypes = [vp, C.POINTER(Scene), C.c_int, C.POINTER(Camera), C.POINTER(Settings),
                                                vp, C.c_size_t, u64, vp, C.POINTER(vp), C.POINTER(vp), vp, C.c_size_t,
                                                C.POINTER(SceneGrad)]
        L.aaa_stage_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.c_int]
        L.aaa_sort_tmp_size.argtypes = [u64, C.POINTER(C.c_size_t)]
        L.aaa_sort_pairs.argtypes = [vp, vp, u64, C.c_int, vp, C.c_size_t, vp]
        L.aaa_measure_peaks.argtypes = [vp, C.c_size_t, C.c_int, vp, C.POINTER(C.c_double)]
        for f in EXPORTS:
            if f not in ("aaa_destroy", "aaa_last_error", "aaa_version"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def check(rc: int):
    if rc != AAA_OK:
        raise AAAError(rc, lib().aaa_last_error().decode(errors="replace"))


def make_camera(cam) -> Camera:
    c = Camera()
    vm = [float(v) for v in __import__("numpy").asarray(cam.viewmat, dtype="float64").reshape(16)]
    for i in range(16):
        c.viewmat[i] = vm[i]
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.width, c.height, c.znear = int(cam.width), int(cam.height), float(cam.znear)
    for i in range(3):
        c.bg[i] = float(cam.bg[i])
    return c


def make_settings(st, extra_flags: int = 0) -> Settings:
    s = Settings()
    s.filter_k = float(st.filter_k)
    s.ray_window = int(st.ray_window)
    flags = extra_flags
    if st.filter_mode == 1:
        flags |= AAA_FILTER_OFF
    elif st.filter_mode == 2:
        flags |= AAA_FILTER_VOLUME
    if not st.tile_cull:
        flags |= AAA_NO_TILE_CULL
    if getattr(st, "subtile_sort", False):
        flags |= AAA_SUBTILE_SORT
    s.flags = flags
    s.alpha_min, s.alpha_max, s.t_min = float(st.alpha_min), float(st.alpha_max), float(st.t_min)
    return s
