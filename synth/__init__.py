"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

The paper evaluates on an unnamed volume data set that is not available
(Sec. 5, Fig. 3, Table 1), so seeded Gaussian-blob volumes stand in for it.
This module only *produces inputs*: cameras, blob volumes, the server-side
ray-cast 2.5D image (RGBA + depth, Sec. 4.1) and random sphere sets for small
tests.  It holds none of the client method's arithmetic (unprojection,
hierarchy construction, sphere tracing, compositing of splats).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, replace

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")

VOLUME_CENTRE = np.array([0.5, 0.5, 0.5])
# World box of the volume: edge 1.5 centred on VOLUME_CENTRE.  With the camera
# 2.0 from the centre this covers ~70% of a 1024^2 source image with splats,
# close to the paper's 623,584 of 1024^2 samples (59.5%, Table 1).
BOX_LO = -0.25
BOX_SIZE = 1.5


def build(force: bool = True) -> str:
    """Compile the C generator with gcc/OpenMP into synth/libsynth.so."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Cam(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("forward", ctypes.c_double * 3),
                ("right", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
                ("tan_half_fov_y", ctypes.c_double), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.syn_make_volume.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.syn_raycast.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_Cam),
                                    ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclass(frozen=True)
class Camera:
    """Pinhole camera: orthonormal basis, vertical half-angle tangent, image size.

    Pixel (x, y) looks along normalize(F + sx R + sy U) with
    sx = ((2x+1)/W - 1) tan(fov/2) W/H and sy = (1 - (2y+1)/H) tan(fov/2);
    row 0 is the top row.
    """
    eye: tuple
    forward: tuple
    right: tuple
    up: tuple
    tan_half_fov_y: float
    width: int
    height: int

    def to_c(self) -> _Cam:
        c = _Cam()
        c.eye[:] = self.eye
        c.forward[:] = self.forward
        c.right[:] = self.right
        c.up[:] = self.up
        c.tan_half_fov_y = self.tan_half_fov_y
        c.width, c.height = self.width, self.height
        return c

    def resized(self, width: int, height: int) -> "Camera":
        return replace(self, width=int(width), height=int(height))


def _rot(axis, deg):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    a = math.radians(deg)
    x, y, z = axis
    c, s = math.cos(a), math.sin(a)
    C = 1.0 - c
    return np.array([[c + x * x * C, x * y * C - z * s, x * z * C + y * s],
                     [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
                     [z * x * C - y * s, z * y * C + x * s, c + z * z * C]])


def source_camera(width: int, height: int, fov_y_deg: float = 45.0, distance: float = 2.0) -> Camera:
    """Source camera on +z at `distance` from the volume centre, looking at it, up +y."""
    eye = VOLUME_CENTRE + distance * np.array([0.0, 0.0, 1.0])
    return Camera(tuple(eye), (0.0, 0.0, -1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0),
                  math.tan(math.radians(fov_y_deg) / 2.0), int(width), int(height))


def rotated_camera(cam: Camera, yaw_deg: float, pitch_deg: float = 0.0,
                   width: int | None = None, height: int | None = None) -> Camera:
    """Orbit `cam` about the volume centre: yaw about +y, then pitch about the yawed right axis."""
    Ry = _rot([0, 1, 0], yaw_deg)
    right1 = Ry @ np.array(cam.right)
    R = _rot(right1, pitch_deg) @ Ry
    eye = VOLUME_CENTRE + R @ (np.array(cam.eye) - VOLUME_CENTRE)
    f, r, u = (R @ np.array(cam.forward), R @ np.array(cam.right), R @ np.array(cam.up))
    return Camera(tuple(eye), tuple(f), tuple(r), tuple(u), cam.tan_half_fov_y,
                  int(width or cam.width), int(height or cam.height))


def blob_params(seed: int, nblobs: int):
    """Blob centres U[0.2,0.8]^3, sigma U[0.03,0.1], amplitude U[0.5,1], drawn in that order."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, size=(nblobs, 3))
    sigmas = rng.uniform(0.03, 0.1, size=nblobs)
    amps = rng.uniform(0.5, 1.0, size=nblobs)
    return centres, sigmas, amps


def make_volume(n: int, nblobs: int, seed: int) -> np.ndarray:
    """float32 [n][n][n] (z, y, x) sum of seeded Gaussian blobs."""
    centres, sigmas, amps = blob_params(seed, nblobs)
    vol = np.empty((n, n, n), dtype=np.float32)
    c = np.ascontiguousarray(centres, dtype=np.float64)
    s = np.ascontiguousarray(sigmas, dtype=np.float64)
    a = np.ascontiguousarray(amps, dtype=np.float64)
    rc = _load().syn_make_volume(n, nblobs, c.ctypes.data, s.ctypes.data, a.ctypes.data, vol.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"syn_make_volume failed ({rc})")
    return vol


def raycast(vol: np.ndarray, cam: Camera):
    """Server-side ray marcher: premultiplied float32 RGBA [H][W][4] and depth float32 [H][W]."""
    vol = np.ascontiguousarray(vol, dtype=np.float32)
    n = vol.shape[0]
    rgba = np.empty((cam.height, cam.width, 4), dtype=np.float32)
    depth = np.empty((cam.height, cam.width), dtype=np.float32)
    c = cam.to_c()
    rc = _load().syn_raycast(vol.ctypes.data, n, BOX_LO, BOX_SIZE, ctypes.byref(c), rgba.ctypes.data, depth.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"syn_raycast failed ({rc})")
    return rgba, depth


# ---------------------------------------------------------------- workloads

@dataclass(frozen=True)
class Workload:
    name: str
    vol_n: int
    nblobs: int
    seed: int
    src_w: int
    src_h: int
    dst_w: int
    dst_h: int
    yaw: float
    pitch: float


# The blob-volume workloads used for parity and measurement.
TINY = Workload("tiny-64x64", 64, 8, 1, 64, 64, 64, 64, 5.0, 0.0)
CLIENT_FRAME = Workload("client-1024sq-to-1920x1080", 256, 64, 2, 1024, 1024, 1920, 1080, 10.0, 3.0)
LARGE = Workload("large-3840x2160", 512, 256, 3, 3840, 2160, 3840, 2160, 15.0, 0.0)
DIFF = Workload("diff-512sq", 64, 8, 1, 512, 512, 512, 512, 5.0, 0.0)


_cache: dict = {}


def source_image(w: Workload):
    """(rgba, depth, src_cam, dst_cam) for a workload; cached per process."""
    key = w
    if key not in _cache:
        vol = make_volume(w.vol_n, w.nblobs, w.seed)
        src = source_camera(w.src_w, w.src_h)
        rgba, depth = raycast(vol, src)
        dst = rotated_camera(src, w.yaw, w.pitch, w.dst_w, w.dst_h)
        _cache[key] = (rgba, depth, src, dst, vol)
    rgba, depth, src, dst, _ = _cache[key]
    return rgba, depth, src, dst


def volume_of(w: Workload) -> np.ndarray:
    source_image(w)
    return _cache[w][4]


# ---------------------------------------------------------------- batched frames

@dataclass(frozen=True)
class BatchFrame:
    index: int
    seed: int
    nblobs: int
    src: int          # square source size
    dst_w: int
    dst_h: int
    yaws: tuple       # one target pose per yaw (degrees)


def batch_frames(n_frames: int = 64, meta_seed: int = 5, vol_n: int = 128,
                 src_sizes=(256, 512, 1024, 2048), dst_sizes=((640, 480), (1280, 720), (1920, 1080))):
    """Client frames of uneven sizes: per frame a source size, a target size, 16-128 blobs
    (seed 5000 + frame) and 1-8 target poses at yaw U[0, 20) degrees, all drawn from `meta_seed`."""
    rng = np.random.default_rng(meta_seed)
    frames = []
    for f in range(n_frames):
        src = int(rng.choice(src_sizes))
        dw, dh = dst_sizes[int(rng.integers(len(dst_sizes)))]
        nblobs = int(rng.integers(16, 129))
        poses = int(rng.integers(1, 9))
        yaws = tuple(float(y) for y in rng.uniform(0.0, 20.0, poses))
        frames.append(BatchFrame(f, 5000 + f, nblobs, src, int(dw), int(dh), yaws))
    return frames


def batch_frame_images(fr: BatchFrame, vol_n: int = 128):
    """(rgba, depth, src_cam, [dst_cams]) of one batched frame."""
    vol = make_volume(vol_n, fr.nblobs, fr.seed)
    src = source_camera(fr.src, fr.src)
    rgba, depth = raycast(vol, src)
    dsts = [rotated_camera(src, y, 0.0, fr.dst_w, fr.dst_h) for y in fr.yaws]
    return rgba, depth, src, dsts


# ---------------------------------------------------------------- small scenes

def random_spheres(n: int, seed: int, centre_lo=0.3, centre_hi=0.7, r_lo=0.01, r_hi=0.06,
                   a_lo=0.3, a_hi=1.0):
    """Random sphere set: centre_radius float32 [n][4], rgba float32 [n][4] (straight rgb + alpha)."""
    rng = np.random.default_rng(seed)
    cr = np.empty((n, 4), dtype=np.float32)
    cr[:, :3] = rng.uniform(centre_lo, centre_hi, size=(n, 3))
    cr[:, 3] = rng.uniform(r_lo, r_hi, size=n)
    col = np.empty((n, 4), dtype=np.float32)
    col[:, :3] = rng.uniform(0.0, 1.0, size=(n, 3))
    col[:, 3] = rng.uniform(a_lo, a_hi, size=n)
    return cr, col


def adversarial_spheres(seed: int):
    """Coincident, nested, equal-depth and duplicate-position spheres."""
    rng = np.random.default_rng(seed)
    base_cr, base_col = random_spheres(48, seed, 0.4, 0.6, 0.02, 0.05)
    extra_cr, extra_col = [], []
    for i in range(0, 16):
        extra_cr.append(base_cr[i].copy())              # exact duplicates (equal keys, equal t)
        extra_col.append(rng.uniform(0, 1, 4).astype(np.float32))
    for i in range(16, 24):
        c = base_cr[i].copy()
        c[3] *= 0.5                                     # nested: same centre, smaller radius
        extra_cr.append(c)
        extra_col.append(rng.uniform(0, 1, 4).astype(np.float32))
    for i in range(24, 32):
        c = base_cr[i].copy()
        c[0] += 1e-7                                    # near-duplicates: identical Morton cell
        extra_cr.append(c)
        extra_col.append(rng.uniform(0, 1, 4).astype(np.float32))
    cr = np.concatenate([base_cr, np.array(extra_cr, dtype=np.float32)])
    col = np.concatenate([base_col, np.array(extra_col, dtype=np.float32)])
    col[:, 3] = np.clip(col[:, 3], 0.2, 1.0)
    return np.ascontiguousarray(cr), np.ascontiguousarray(col)


def to_half_rgba(col: np.ndarray) -> np.ndarray:
    """Round straight RGBA to float16 (round-to-nearest-even) for half-precision sphere colours."""
    return np.ascontiguousarray(col.astype(np.float16))
