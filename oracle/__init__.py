"""FP64 CPU oracle for the client-side splat ray-tracing path (arXiv 2006.14726).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg are the only users.  The product path never
imports this package; it shares no code with the GPU library.

Everything is computed in double precision by ``oracle.c`` (plain C, OpenMP
over pixels), brute force: every ray against every sphere, hits sorted by
(t0, id), composited in order.  This module only marshals arrays:

* ``unproject``  Sec. 4.1, Eq. 1 (p = o + d t_i), footprint radius, compaction
* ``render``     Sec. 4.1 / Fig. 2: spheres traced from a new camera,
                 composited front to back with an alpha stop; or spheroids
                 (samples smeared along their source ray, Sec. 7)
* ``unproject_spheroids``  those spheroids from a depth interval (Sec. 7)
* ``grad``       analytic gradient of a per-pixel loss through ``render``
* ``half_bits``  double -> binary16 with round-to-nearest-even
* ``raymarch``   the server stage before the path (Sec. 4.1): volume ray
                 marcher writing premultiplied colour and a representative depth
* ``encode``, ``decode``  the wire format: 64 bits per sample (quantised
                 position + radius), 32 bits per colour (Sec. 4.1, Sec. 6)
* ``accumulate`` temporal accumulation across frames (Sec. 7): the new
                 frame's samples, then the history samples whose grid cell the
                 frame does not occupy and that are not too old
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

MODE_CONSTANT = 0
MODE_SOFT = 1

FLAG_GRAZE = 1
FLAG_KNIFE = 2
FLAG_MULTI_KNIFE = 4


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into oracle/liboracle.so (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Cam(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("forward", ctypes.c_double * 3),
                ("right", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
                ("tan_half_fov_y", ctypes.c_double), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32)]


def _cam(c) -> _Cam:
    out = _Cam()
    out.eye[:] = [float(v) for v in c.eye]
    out.forward[:] = [float(v) for v in c.forward]
    out.right[:] = [float(v) for v in c.right]
    out.up[:] = [float(v) for v in c.up]
    out.tan_half_fov_y = float(c.tan_half_fov_y)
    out.width, out.height = int(c.width), int(c.height)
    return out


_lib = None
_P = ctypes.c_void_p


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        lib.orc_half_bits.argtypes = [ctypes.c_double]
        lib.orc_half_bits.restype = ctypes.c_uint16
        lib.orc_unproject.argtypes = [ctypes.POINTER(_Cam), _P, _P, ctypes.c_double, _P, _P, _P, _P]
        lib.orc_unproject.restype = ctypes.c_int64
        lib.orc_render.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(_Cam), ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, _P, ctypes.c_int64, _P, _P, _P, _P, _P, _P]
        lib.orc_render.restype = ctypes.c_int
        lib.orc_grad.argtypes = [_P, ctypes.c_int64, ctypes.POINTER(_Cam), ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int, _P, _P]
        lib.orc_grad.restype = ctypes.c_int
        lib.orc_sphere_test.argtypes = [_P, _P, _P, ctypes.c_double, ctypes.c_double, _P]
        lib.orc_sphere_test.restype = ctypes.c_int
        lib.orc_pixels_near.argtypes = [ctypes.POINTER(_Cam), _P, ctypes.c_double, _P, ctypes.c_int64]
        lib.orc_pixels_near.restype = ctypes.c_int64
        lib.orc_volume_sample.argtypes = [_P, ctypes.c_int32, _P]
        lib.orc_volume_sample.restype = ctypes.c_double
        lib.orc_raymarch.argtypes = [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_Cam),
                                     ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, _P, ctypes.c_int64, _P]
        lib.orc_unproject_policy.argtypes = [ctypes.POINTER(_Cam), _P, _P, _P, ctypes.c_int32, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P]
        lib.orc_spheroid_test.argtypes = [_P, _P, _P, ctypes.c_double, _P, ctypes.c_double, ctypes.c_double, _P]
        lib.orc_spheroid_test.restype = ctypes.c_int
        lib.orc_render_axis.argtypes = [_P, _P, ctypes.c_int64, ctypes.POINTER(_Cam), ctypes.c_double,
                                        ctypes.c_double, ctypes.c_int, _P, ctypes.c_int64, _P, _P, _P, _P, _P, _P]
        lib.orc_render_axis.restype = ctypes.c_int
        lib.orc_unproject_policy.restype = ctypes.c_int64
        lib.orc_raymarch.restype = ctypes.c_int
        lib.orc_encode_position.argtypes = [_P, ctypes.c_double, _P, ctypes.c_double, ctypes.c_double]
        lib.orc_encode_position.restype = ctypes.c_uint64
        lib.orc_encode_colour.argtypes = [_P]
        lib.orc_encode_colour.restype = ctypes.c_uint32
        lib.orc_encode.argtypes = [_P, _P, ctypes.c_int64, _P, ctypes.c_double, ctypes.c_double, _P, _P]
        lib.orc_encode.restype = None
        lib.orc_decode.argtypes = [_P, _P, ctypes.c_int64, _P, ctypes.c_double, ctypes.c_double, _P, _P]
        lib.orc_decode.restype = None
        lib.orc_accumulate.argtypes = [_P, ctypes.c_int64, _P, _P, ctypes.c_int64, _P, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_int32, _P]
        lib.orc_accumulate.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def half_bits(values) -> np.ndarray:
    """binary16 bit patterns of float64 values, round-to-nearest-even."""
    v = np.asarray(values, dtype=np.float64).ravel()
    lib = _load()
    return np.array([lib.orc_half_bits(float(x)) for x in v], dtype=np.uint16)


def unproject(cam, rgba: np.ndarray, depth: np.ndarray, radius_scale: float, half: bool):
    """Eq. 1 unprojection of a premultiplied RGBA + depth image.

    Returns (centre_radius float32 [N][4], colour [N][4] float16 or float32
    straight RGBA, src_index uint32 [N]).
    """
    H, W = int(cam.height), int(cam.width)
    rgba = np.ascontiguousarray(rgba, dtype=np.float32).reshape(H, W, 4)
    depth = np.ascontiguousarray(depth, dtype=np.float32).reshape(H, W)
    cap = H * W
    cr = np.zeros((cap, 4), dtype=np.float32)
    col32 = None if half else np.zeros((cap, 4), dtype=np.float32)
    col16 = np.zeros((cap, 4), dtype=np.uint16) if half else None
    idx = np.zeros(cap, dtype=np.uint32)
    c = _cam(cam)
    n = _load().orc_unproject(ctypes.byref(c), rgba.ctypes.data, depth.ctypes.data, float(radius_scale),
                              cr.ctypes.data, _ptr(col32), _ptr(col16), idx.ctypes.data)
    col = col16.view(np.float16) if half else col32
    return cr[:n].copy(), col[:n].copy(), idx[:n].copy()


RADIUS_FOOTPRINT, RADIUS_OPACITY, RADIUS_INTERVAL, RADIUS_SPHEROID = 0, 1, 2, 3


def unproject_policy(cam, rgba: np.ndarray, depth: np.ndarray, mode: int, radius_scale: float = 1.0,
                     opacity_floor: float = 0.05, interval_scale: float = 1.0, interval: np.ndarray | None = None,
                     half: bool = True):
    """Unprojection with a radius policy (Sec. 7): footprint, opacity (r = s fp sqrt(max(A, floor))) or
    interval (centre at the depth interval's midpoint, r = max(s fp, kappa half-length)).
    Returns (centre_radius float32 [N][4], colour [N][4] float16 or float32, src_index uint32 [N])."""
    H, W = int(cam.height), int(cam.width)
    rgba = np.ascontiguousarray(rgba, dtype=np.float32).reshape(H, W, 4)
    depth = np.ascontiguousarray(depth, dtype=np.float32).reshape(H, W)
    itv = None
    if mode == RADIUS_INTERVAL:
        itv = np.ascontiguousarray(interval, dtype=np.float32).reshape(H, W, 2)
    cap = H * W
    cr = np.zeros((cap, 4), dtype=np.float32)
    col32 = None if half else np.zeros((cap, 4), dtype=np.float32)
    col16 = np.zeros((cap, 4), dtype=np.uint16) if half else None
    idx = np.zeros(cap, dtype=np.uint32)
    c = _cam(cam)
    # the floor and kappa are float parameters of the GPU call: use their float values
    assert mode != RADIUS_SPHEROID, "unproject_spheroids returns the axes too"
    n = _load().orc_unproject_policy(ctypes.byref(c), rgba.ctypes.data, depth.ctypes.data, _ptr(itv), int(mode),
                                     float(np.float32(radius_scale)), float(np.float32(opacity_floor)),
                                     float(np.float32(interval_scale)), cr.ctypes.data, _ptr(col32), _ptr(col16),
                                     idx.ctypes.data, None)
    col = col16.view(np.float16) if half else col32
    return cr[:n].copy(), col[:n].copy(), idx[:n].copy()


def unproject_spheroids(cam, rgba: np.ndarray, depth: np.ndarray, interval: np.ndarray, radius_scale: float = 1.0,
                        interval_scale: float = 1.0, half: bool = True):
    """Samples smeared along their source ray over the depth interval (Sec. 7): prolate spheroids centred at the
    interval's midpoint, radius s fp(t_c) across the ray, half-length max(r, kappa half-interval) along it.
    Returns (centre_radius float32 [N][4], colour [N][4], src_index uint32 [N], axis float32 [N][4] = (u, h))."""
    H, W = int(cam.height), int(cam.width)
    rgba = np.ascontiguousarray(rgba, dtype=np.float32).reshape(H, W, 4)
    depth = np.ascontiguousarray(depth, dtype=np.float32).reshape(H, W)
    itv = np.ascontiguousarray(interval, dtype=np.float32).reshape(H, W, 2)
    cap = H * W
    cr = np.zeros((cap, 4), dtype=np.float32)
    col32 = None if half else np.zeros((cap, 4), dtype=np.float32)
    col16 = np.zeros((cap, 4), dtype=np.uint16) if half else None
    idx = np.zeros(cap, dtype=np.uint32)
    ax = np.zeros((cap, 4), dtype=np.float32)
    c = _cam(cam)
    n = _load().orc_unproject_policy(ctypes.byref(c), rgba.ctypes.data, depth.ctypes.data, itv.ctypes.data,
                                     RADIUS_SPHEROID, float(np.float32(radius_scale)), 1.0,
                                     float(np.float32(interval_scale)), cr.ctypes.data, _ptr(col32), _ptr(col16),
                                     idx.ctypes.data, ax.ctypes.data)
    col = col16.view(np.float16) if half else col32
    return cr[:n].copy(), col[:n].copy(), idx[:n].copy(), ax[:n].copy()


def sphere_table(centre_radius: np.ndarray, colour: np.ndarray) -> np.ndarray:
    """Exact widening of the stored sphere values to the oracle's [N][8] float64 table."""
    cr = np.asarray(centre_radius).reshape(-1, 4).astype(np.float64)
    col = np.asarray(colour).reshape(-1, 4).astype(np.float64)
    return np.ascontiguousarray(np.concatenate([cr, col], axis=1))


def render_table(table: np.ndarray, cam, alpha_stop: float = 0.99, t_max: float = np.inf,
                 mode: int = MODE_CONSTANT, pixels=None, axis=None):
    """Brute-force render from an [N][8] float64 sphere table (cx cy cz r kr kg kb a); with `axis` ([N][4] u, h)
    the samples are prolate spheroids (constant alpha only)."""
    table = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 8)
    ax = None if axis is None else np.ascontiguousarray(np.asarray(axis).reshape(-1, 4).astype(np.float64))
    assert ax is None or ax.shape[0] == table.shape[0]
    if pixels is None:
        pix = None
        npix = int(cam.width) * int(cam.height)
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64).ravel()
        npix = pix.size
    out = np.zeros((npix, 4), dtype=np.float64)
    alt = np.zeros((npix, 4), dtype=np.float64)
    n = np.zeros(npix, dtype=np.int32)
    nalt = np.zeros(npix, dtype=np.int32)
    flags = np.zeros(npix, dtype=np.int32)
    sig = np.zeros(npix, dtype=np.uint64)
    c = _cam(cam)
    if ax is None:
        rc = _load().orc_render(table.ctypes.data, table.shape[0], ctypes.byref(c), float(alpha_stop), float(t_max),
                                int(mode), _ptr(pix), npix, out.ctypes.data, n.ctypes.data, flags.ctypes.data,
                                alt.ctypes.data, nalt.ctypes.data, sig.ctypes.data)
    else:
        rc = _load().orc_render_axis(table.ctypes.data, ax.ctypes.data, table.shape[0], ctypes.byref(c),
                                     float(alpha_stop), float(t_max), int(mode), _ptr(pix), npix, out.ctypes.data,
                                     n.ctypes.data, flags.ctypes.data, alt.ctypes.data, nalt.ctypes.data,
                                     sig.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_render failed ({rc})")
    return {"rgba": out, "n": n, "flags": flags, "alt_rgba": alt, "alt_n": nalt, "sig": sig}


def render(centre_radius, colour, cam, alpha_stop: float = 0.99, t_max: float = np.inf,
           mode: int = MODE_CONSTANT, pixels=None, axis=None):
    """Brute-force FP64 render of stored spheres (float32 centre/radius, float16/32 colour), or of spheroids
    with the stored axes (float32 [N][4]: unit axis, half-length along it)."""
    return render_table(sphere_table(centre_radius, colour), cam, alpha_stop, t_max, mode, pixels, axis)


def grad_table(table: np.ndarray, cam, grad_rgba: np.ndarray, alpha_stop: float = 0.99,
               t_max: float = np.inf, mode: int = MODE_SOFT) -> np.ndarray:
    """dL/d(cx cy cz r kr kg kb a) [N][8] for L = sum(grad_rgba * I)."""
    table = np.ascontiguousarray(table, dtype=np.float64).reshape(-1, 8)
    g = np.ascontiguousarray(grad_rgba, dtype=np.float64).reshape(-1, 4)
    assert g.shape[0] == int(cam.width) * int(cam.height)
    out = np.zeros_like(table)
    c = _cam(cam)
    rc = _load().orc_grad(table.ctypes.data, table.shape[0], ctypes.byref(c), float(alpha_stop), float(t_max),
                          int(mode), g.ctypes.data, out.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"orc_grad failed ({rc})")
    return out


def sphere_test(o, d, c, r: float, t_max: float = np.inf):
    """One ray against one sphere: (hit, t0, q, disc, v[3], b)."""
    o = np.ascontiguousarray(o, dtype=np.float64)
    d = np.ascontiguousarray(d, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(7, dtype=np.float64)
    hit = _load().orc_sphere_test(o.ctypes.data, d.ctypes.data, c.ctypes.data, float(r), float(t_max),
                                  out.ctypes.data)
    return bool(hit), out[0], out[1], out[2], out[3:6].copy(), out[6]


def spheroid_test(o, d, c, r: float, u, h: float, t_max: float = np.inf):
    """One ray against one prolate spheroid: (hit, t0, disc, t_mid, qq)."""
    a = [np.ascontiguousarray(v, dtype=np.float64) for v in (o, d, c, u)]
    out = np.zeros(4, dtype=np.float64)
    hit = _load().orc_spheroid_test(a[0].ctypes.data, a[1].ctypes.data, a[2].ctypes.data, float(r), a[3].ctypes.data,
                                    float(h), float(t_max), out.ctypes.data)
    return bool(hit), out[0], out[1], out[2], out[3]


def pixels_near(cam, centre, radius: float) -> np.ndarray:
    """Row-major ids of pixels whose ray passes within `radius` of `centre` (in front of the eye)."""
    c = _cam(cam)
    ctr = np.ascontiguousarray(centre, dtype=np.float64)
    cap = int(cam.width) * int(cam.height)
    out = np.zeros(cap, dtype=np.int64)
    n = _load().orc_pixels_near(ctypes.byref(c), ctr.ctypes.data, float(radius), out.ctypes.data, cap)
    return out[:n].copy()


# server stage defaults: the workloads' transfer and depth rules
MARCH_STEP = 0.5          # voxels between samples
MARCH_ALPHA_SCALE = 0.05  # sample alpha = clamp(0.05 v, 0, 1)
MARCH_DEPTH_ALPHA = 0.5   # depth = first sample at which A >= 0.5
MARCH_STOP_ALPHA = 0.999  # stop after the sample at which A >= 0.999
MARCH_INTERVAL_LO = 0.25  # depth interval: first sample at which A >= 0.25 ...
MARCH_INTERVAL_HI = 0.75  # ... to the first at which A >= 0.75 (or the last sample taken)


def volume_sample(vol: np.ndarray, p) -> float:
    """Trilinear (clamp-to-edge) value of vol [n][n][n] (z, y, x) at normalised position p."""
    v = np.ascontiguousarray(vol, dtype=np.float32)
    q = np.ascontiguousarray(p, dtype=np.float64)
    return float(_load().orc_volume_sample(v.ctypes.data, int(v.shape[0]), q.ctypes.data))


def raymarch(vol: np.ndarray, box_lo: float, box_size: float, cam, pixels=None, step: float = MARCH_STEP,
             alpha_scale: float = MARCH_ALPHA_SCALE, depth_alpha: float = MARCH_DEPTH_ALPHA,
             stop_alpha: float = MARCH_STOP_ALPHA, interval_lo: float = MARCH_INTERVAL_LO,
             interval_hi: float = MARCH_INTERVAL_HI) -> dict:
    """Server ray marcher in double precision.  Returns {"rgba": [k][4] premultiplied, "depth": [k],
    "interval": [k][2] (t_lo, t_hi)} (float64) for all pixels (row-major) or the given pixel indices."""
    v = np.ascontiguousarray(vol, dtype=np.float32)
    n = int(v.shape[0])
    assert v.shape == (n, n, n)
    c = _cam(cam)
    if pixels is None:
        count, pix = int(cam.width) * int(cam.height), None
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        count = len(pix)
    out = np.zeros((count, 7), dtype=np.float64)
    _load().orc_raymarch(v.ctypes.data, n, float(box_lo), float(box_size), ctypes.byref(c), float(step),
                         float(alpha_scale), float(depth_alpha), float(stop_alpha), float(interval_lo),
                         float(interval_hi), None if pix is None else pix.ctypes.data, count, out.ctypes.data)
    return {"rgba": out[:, :4].copy(), "depth": out[:, 4].copy(), "interval": out[:, 5:7].copy()}


CODEC_POS_BITS = 18      # per axis
CODEC_R_STEPS = 64       # radius codes per octave around r_unit (code 512 = r_unit)


def encode(centre_radius: np.ndarray, rgba: np.ndarray, box_lo, box_size: float, r_unit: float):
    """Spheres -> (uint64 [n] position+radius words, uint32 [n] RGBA8 colours)."""
    cr = np.ascontiguousarray(centre_radius, dtype=np.float32).reshape(-1, 4)
    col = np.ascontiguousarray(rgba, dtype=np.float64).reshape(-1, 4)
    n = cr.shape[0]
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(box_lo, dtype=np.float64), (3,)))
    pos = np.zeros(n, dtype=np.uint64)
    out = np.zeros(n, dtype=np.uint32)
    _load().orc_encode(cr.ctypes.data, col.ctypes.data, n, lo.ctypes.data, float(box_size), float(r_unit),
                       pos.ctypes.data, out.ctypes.data)
    return pos, out


def decode(pos: np.ndarray, col: np.ndarray, box_lo, box_size: float, r_unit: float):
    """(words, colours) -> (centre_radius float32 [n][4], rgba float32 [n][4])."""
    p = np.ascontiguousarray(pos, dtype=np.uint64)
    c = np.ascontiguousarray(col, dtype=np.uint32)
    n = p.shape[0]
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(box_lo, dtype=np.float64), (3,)))
    cr = np.zeros((n, 4), dtype=np.float32)
    rgba = np.zeros((n, 4), dtype=np.float32)
    _load().orc_decode(p.ctypes.data, c.ctypes.data, n, lo.ctypes.data, float(box_size), float(r_unit),
                       cr.ctypes.data, rgba.ctypes.data)
    return cr, rgba


def encode_position(c, r: float, box_lo, box_size: float, r_unit: float) -> int:
    cc = np.ascontiguousarray(c, dtype=np.float64)
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(box_lo, dtype=np.float64), (3,)))
    return int(_load().orc_encode_position(cc.ctypes.data, float(r), lo.ctypes.data, float(box_size), float(r_unit)))


def encode_colour(k) -> int:
    kk = np.ascontiguousarray(k, dtype=np.float64)
    return int(_load().orc_encode_colour(kk.ctypes.data))


def accumulate_survivors(frame_cr: np.ndarray, hist_cr: np.ndarray, hist_age: np.ndarray, box_lo, box_size: float,
                         grid: int, max_age: int) -> np.ndarray:
    """Indices (ascending) of the history samples that survive the merge with a new frame."""
    f = np.ascontiguousarray(frame_cr, dtype=np.float32).reshape(-1, 4)
    h = np.ascontiguousarray(hist_cr, dtype=np.float32).reshape(-1, 4)
    age = np.ascontiguousarray(hist_age, dtype=np.uint8).reshape(-1)
    assert age.shape[0] == h.shape[0]
    lo = np.ascontiguousarray(np.broadcast_to(np.asarray(box_lo, dtype=np.float64), (3,)))
    kept = np.zeros(max(h.shape[0], 1), dtype=np.int64)
    n = _load().orc_accumulate(f.ctypes.data, f.shape[0], h.ctypes.data, age.ctypes.data, h.shape[0], lo.ctypes.data,
                               float(box_size), int(grid), int(max_age), kept.ctypes.data)
    if n < 0:
        raise RuntimeError("orc_accumulate: out of memory")
    return kept[:n].copy()


def accumulate(frame: dict, history: dict, box_lo, box_size: float, grid: int, max_age: int,
               capacity: int | None = None) -> dict:
    """Merged sample set of a new frame and the history (Sec. 7, temporal accumulation).

    ``frame`` holds ``cr`` (float32 [n][4]) and ``rgba`` ([n][4], any dtype),
    optionally ``src`` (uint32 [n]); ``history`` the same plus ``age`` (uint8
    [m]).  The result: frame samples with age 0, then the surviving history
    samples with age + 1, cut to ``capacity``."""
    keep = accumulate_survivors(frame["cr"], history["cr"], history["age"], box_lo, box_size, grid, max_age)
    out = {
        "cr": np.concatenate([np.asarray(frame["cr"]).reshape(-1, 4), np.asarray(history["cr"]).reshape(-1, 4)[keep]]),
        "rgba": np.concatenate([np.asarray(frame["rgba"]).reshape(-1, 4),
                                np.asarray(history["rgba"]).reshape(-1, 4)[keep]]),
        "age": np.concatenate([np.zeros(len(frame["cr"]), dtype=np.uint8),
                               (np.asarray(history["age"], dtype=np.int32)[keep] + 1).astype(np.uint8)]),
    }
    if "src" in frame and "src" in history:
        out["src"] = np.concatenate([np.asarray(frame["src"]), np.asarray(history["src"])[keep]]).astype(np.uint32)
    if capacity is not None:
        out = {k: v[:capacity] for k, v in out.items()}
    out["kept"] = keep
    return out
