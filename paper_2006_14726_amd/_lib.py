"""ctypes view of libsplat.so (include/splat.h).  Marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsplat.so")

SPLAT_OK, SPLAT_EINVAL, SPLAT_ENOSPC, SPLAT_ENODEV, SPLAT_EHIP, SPLAT_EUNSUPPORTED = range(6)
SPLAT_F32, SPLAT_F16 = 0, 1
SPLAT_ALPHA_CONSTANT, SPLAT_ALPHA_SOFT = 0, 1
SPLAT_WALK_LANE, SPLAT_WALK_PACKET = 0, 1
SPLAT_RADIUS_FOOTPRINT, SPLAT_RADIUS_OPACITY, SPLAT_RADIUS_INTERVAL, SPLAT_RADIUS_SPHEROID = 0, 1, 2, 3
SPLAT_STATUS_CORRUPT, SPLAT_STATUS_STACK = 1, 2
SPLAT_BATCH_GRID = -1
SPLAT_BVH_STATUS_OFFSET = 56
SPLAT_OP_UNPROJECT, SPLAT_OP_BUILD, SPLAT_OP_TRACE, SPLAT_OP_BACKWARD, SPLAT_OP_BATCHED, SPLAT_OP_ACCUMULATE = range(6)

# every symbol include/splat.h declares
EXPORTS = ["splat_workspace_bytes", "splat_bvh_bytes", "splat_raymarch", "splat_encode_samples",
           "splat_decode_samples", "splat_accumulate", "splat_unproject", "splat_unproject_policy", "splat_build_bvh", "splat_trace", "splat_trace_backward",
           "splat_trace_batched", "splat_last_error", "splat_version", "splat_trace_noalloc",
           "splat_trace_noalloc_max_bytes", "splat_bvh_status_word", "splat_build_bvh_from_samples"]

_P = ctypes.c_void_p


class splat_camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("forward", ctypes.c_double * 3), ("right", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("tan_half_fov_y", ctypes.c_double), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32)]


class splat_spheres(ctypes.Structure):
    _fields_ = [("centre_radius", _P), ("rgba", _P), ("rgba_dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("src_index", _P), ("count", _P), ("capacity", ctypes.c_uint32), ("axis", _P)]


class splat_bvh(ctypes.Structure):
    _fields_ = [("mem", _P), ("capacity", ctypes.c_uint32)]


class splat_trace_opts(ctypes.Structure):
    _fields_ = [("alpha_stop", ctypes.c_float), ("mode", ctypes.c_int32), ("t_max", ctypes.c_double),
                ("kbuf", ctypes.c_int32), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("walk", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("event_begin", _P), ("event_end", _P)]


class splat_volume(ctypes.Structure):
    _fields_ = [("data", _P), ("n", ctypes.c_int32), ("box_lo", ctypes.c_double), ("box_size", ctypes.c_double)]


class splat_march_opts(ctypes.Structure):
    _fields_ = [("step", ctypes.c_double), ("alpha_scale", ctypes.c_double), ("depth_alpha", ctypes.c_double),
                ("stop_alpha", ctypes.c_double), ("interval_lo", ctypes.c_double), ("interval_hi", ctypes.c_double)]


class splat_radius_policy(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("radius_scale", ctypes.c_float), ("opacity_floor", ctypes.c_float),
                ("interval_scale", ctypes.c_float)]


class splat_codec(ctypes.Structure):
    _fields_ = [("box_lo", ctypes.c_double * 3), ("box_size", ctypes.c_double), ("r_unit", ctypes.c_double)]


class splat_accum_opts(ctypes.Structure):
    _fields_ = [("box_lo", ctypes.c_double * 3), ("box_size", ctypes.c_double), ("grid", ctypes.c_int32),
                ("max_age", ctypes.c_int32)]


class splat_grads(ctypes.Structure):
    _fields_ = [("d_rgb", _P), ("d_alpha", _P), ("d_radius", _P), ("d_centre", _P)]


class splat_batch_job(ctypes.Structure):
    _fields_ = [("bvh_mem", _P), ("centre_radius", _P), ("rgba", _P), ("rgba_dtype", ctypes.c_int32),
                ("bvh_capacity", ctypes.c_uint32), ("camera", splat_camera), ("out_rgba", _P), ("out_hits", _P)]


class SplatError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"splat error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree libsplat.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2006_14726_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        lib.splat_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32, ctypes.c_int32]
        lib.splat_workspace_bytes.restype = ctypes.c_size_t
        lib.splat_bvh_bytes.argtypes = [ctypes.c_uint32]
        lib.splat_bvh_bytes.restype = ctypes.c_size_t
        lib.splat_unproject.argtypes = [ctypes.POINTER(splat_camera), _P, _P, ctypes.c_float,
                                        ctypes.POINTER(splat_spheres), _P, ctypes.c_size_t, _P]
        lib.splat_build_bvh.argtypes = [ctypes.POINTER(splat_spheres), ctypes.POINTER(splat_bvh), ctypes.c_int32, _P,
                                        ctypes.c_size_t, _P]
        lib.splat_trace.argtypes = [ctypes.POINTER(splat_bvh), ctypes.POINTER(splat_spheres),
                                    ctypes.POINTER(splat_camera), ctypes.POINTER(splat_trace_opts), _P, _P, _P,
                                    ctypes.c_size_t, _P]
        lib.splat_trace_noalloc.argtypes = [ctypes.POINTER(splat_bvh), ctypes.POINTER(splat_spheres),
                                            ctypes.POINTER(splat_camera), ctypes.POINTER(splat_trace_opts), _P, _P, _P]
        lib.splat_trace_noalloc_max_bytes.argtypes = []
        lib.splat_trace_noalloc_max_bytes.restype = ctypes.c_size_t
        lib.splat_trace_backward.argtypes = [ctypes.POINTER(splat_bvh), ctypes.POINTER(splat_spheres),
                                             ctypes.POINTER(splat_camera), ctypes.POINTER(splat_trace_opts), _P, _P,
                                             ctypes.POINTER(splat_grads), _P, ctypes.c_size_t, _P]
        lib.splat_trace_batched.argtypes = [_P, _P, ctypes.c_int32, ctypes.c_uint32, ctypes.POINTER(splat_trace_opts),
                                            ctypes.c_int32, _P, ctypes.c_size_t, _P]
        lib.splat_last_error.argtypes = []
        lib.splat_last_error.restype = ctypes.c_char_p
        lib.splat_version.argtypes = []
        lib.splat_version.restype = ctypes.c_int
        lib.splat_bvh_status_word.argtypes = [ctypes.POINTER(splat_bvh)]
        lib.splat_bvh_status_word.restype = ctypes.c_void_p
        lib.splat_raymarch.argtypes = [ctypes.POINTER(splat_volume), ctypes.POINTER(splat_camera),
                                       ctypes.POINTER(splat_march_opts), _P, _P, _P, _P]
        lib.splat_unproject_policy.argtypes = [ctypes.POINTER(splat_camera), _P, _P, _P,
                                               ctypes.POINTER(splat_radius_policy), ctypes.POINTER(splat_spheres), _P,
                                               ctypes.c_size_t, _P]
        lib.splat_encode_samples.argtypes = [ctypes.POINTER(splat_spheres), ctypes.POINTER(splat_codec), _P, _P, _P]
        lib.splat_decode_samples.argtypes = [_P, _P, _P, ctypes.POINTER(splat_codec), ctypes.POINTER(splat_spheres),
                                             _P]
        lib.splat_build_bvh_from_samples.argtypes = [_P, _P, _P, ctypes.POINTER(splat_codec),
                                                     ctypes.POINTER(splat_spheres), ctypes.POINTER(splat_bvh), _P,
                                                     ctypes.c_size_t, _P]
        lib.splat_accumulate.argtypes = [ctypes.POINTER(splat_spheres), ctypes.POINTER(splat_spheres), _P,
                                         ctypes.POINTER(splat_accum_opts), ctypes.POINTER(splat_spheres), _P, _P,
                                         ctypes.c_size_t, _P]
        for name in ("splat_raymarch", "splat_encode_samples", "splat_decode_samples", "splat_accumulate",
                     "splat_unproject", "splat_unproject_policy", "splat_build_bvh", "splat_trace", "splat_trace_noalloc",
                     "splat_trace_backward",
                     "splat_trace_batched"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def check(code: int) -> None:
    if code != SPLAT_OK:
        raise SplatError(code, load().splat_last_error().decode(errors="replace"))


def camera_struct(cam) -> splat_camera:
    c = splat_camera()
    c.eye[:] = [float(v) for v in cam.eye]
    c.forward[:] = [float(v) for v in cam.forward]
    c.right[:] = [float(v) for v in cam.right]
    c.up[:] = [float(v) for v in cam.up]
    c.tan_half_fov_y = float(cam.tan_half_fov_y)
    c.width, c.height = int(cam.width), int(cam.height)
    return c
