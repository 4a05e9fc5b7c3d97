"""Torch-facing wrappers of the C ABI: tensors in, tensors out.

Torch only provides device memory and the current stream; every step runs
in the HIP kernels of libsplat.so.  Nothing here synchronises unless a
function says so.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field

import torch

from . import _lib


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _require_cuda(t: torch.Tensor, name: str, dtype=None, contiguous=True):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if contiguous and not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


_workspaces: dict = {}
# Buffers a larger request replaced.  A captured HIP graph keeps the raw
# address of the buffer it was recorded with, so a replaced buffer is never
# freed: a replay then still writes memory that it owns.
_retired: list = []


def workspace(nbytes: int, device, tag: str) -> torch.Tensor:
    """Grow-only scratch buffer per (device, tag), shared by the eager calls of
    this process.  Calls on one stream run in order, so sharing is safe there;
    a caller that needs a buffer of its own passes `ws=` to the wrappers."""
    key = (str(device), tag)
    ws = _workspaces.get(key)
    if ws is None or ws.numel() < nbytes:
        if ws is not None:
            _retired.append(ws)
        ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _workspaces[key] = ws
    return ws


def _own_ws(ws: torch.Tensor | None, nbytes: int, device, tag: str) -> torch.Tensor:
    """The caller's workspace if given (checked for size), else the shared one."""
    if ws is None:
        return workspace(nbytes, device, tag)
    _require_cuda(ws, "ws", torch.uint8)
    if ws.numel() < nbytes:
        raise ValueError(f"ws holds {ws.numel()} bytes, {tag} needs {nbytes}")
    return ws


@dataclass
class Spheres:
    """Sphere set in device memory (capacity slots, `count` used)."""
    centre_radius: torch.Tensor            # float32 [cap, 4]
    rgba: torch.Tensor                     # float16 or float32 [cap, 4], straight colour + alpha
    count: torch.Tensor                    # int32 [1] on the device
    src_index: torch.Tensor | None = None  # int32 [cap]
    axis: torch.Tensor | None = None       # float32 [cap, 4]: spheroids' unit axis and half-length (None: spheres)

    @property
    def capacity(self) -> int:
        return self.centre_radius.shape[0]

    @property
    def half(self) -> bool:
        return self.rgba.dtype == torch.float16

    def struct(self) -> _lib.splat_spheres:
        s = _lib.splat_spheres()
        s.centre_radius = self.centre_radius.data_ptr()
        s.rgba = self.rgba.data_ptr()
        s.rgba_dtype = _lib.SPLAT_F16 if self.half else _lib.SPLAT_F32
        s.src_index = None if self.src_index is None else self.src_index.data_ptr()
        s.count = self.count.data_ptr()
        s.capacity = self.capacity
        s.axis = None if self.axis is None else self.axis.data_ptr()
        return s

    def n(self) -> int:
        """Number of spheres (reads the device count: synchronises)."""
        return int(self.count.item())


def spheres_from_tensors(centre_radius: torch.Tensor, rgba: torch.Tensor, axis: torch.Tensor | None = None) -> Spheres:
    """Wrap existing [N, 4] tensors as a sphere set of N spheres (or of N spheroids with `axis` [N, 4])."""
    _require_cuda(centre_radius, "centre_radius", torch.float32)
    _require_cuda(rgba, "rgba")
    if rgba.dtype not in (torch.float16, torch.float32):
        raise ValueError("rgba must be float16 or float32")
    n = centre_radius.shape[0]
    if centre_radius.shape != (n, 4) or rgba.shape != (n, 4) or n == 0:
        raise ValueError("centre_radius and rgba must both be [N, 4] with N >= 1")
    if axis is not None:
        _require_cuda(axis, "axis", torch.float32)
        if axis.shape != (n, 4):
            raise ValueError("axis must be [N, 4]")
    count = torch.full((1,), n, dtype=torch.int32, device=centre_radius.device)
    return Spheres(centre_radius, rgba, count, axis=axis)


def alloc_spheres(capacity: int, device, half: bool = True, spheroids: bool = False) -> Spheres:
    return Spheres(torch.empty((capacity, 4), dtype=torch.float32, device=device),
                   torch.empty((capacity, 4), dtype=torch.float16 if half else torch.float32, device=device),
                   torch.zeros((1,), dtype=torch.int32, device=device),
                   torch.empty((capacity,), dtype=torch.int32, device=device),
                   torch.empty((capacity, 4), dtype=torch.float32, device=device) if spheroids else None)


def raymarch(volume: torch.Tensor, box_lo: float, box_size: float, cam, step: float = 0.5,
             alpha_scale: float = 0.05, depth_alpha: float = 0.5, stop_alpha: float = 0.999,
             out_rgba: torch.Tensor | None = None, out_depth: torch.Tensor | None = None,
             with_interval: bool = False, interval_lo: float = 0.25, interval_hi: float = 0.75,
             out_interval: torch.Tensor | None = None):
    """Server stage (splat_raymarch): ray-march the float32 volume [n, n, n] (z, y, x) filling the cube
    [box_lo, box_lo + box_size]^3.  Returns (premultiplied rgba [H, W, 4], depth [H, W]), the input of
    `unproject`, and with `with_interval` also the depth interval [H, W, 2] (t_lo, t_hi)."""
    _require_cuda(volume, "volume", torch.float32)
    n = int(volume.shape[0])
    if tuple(volume.shape) != (n, n, n):
        raise ValueError("volume must be [n, n, n]")
    H, W = int(cam.height), int(cam.width)
    if out_rgba is None:
        out_rgba = torch.empty((H, W, 4), dtype=torch.float32, device=volume.device)
    if out_depth is None:
        out_depth = torch.empty((H, W), dtype=torch.float32, device=volume.device)
    _require_cuda(out_rgba, "out_rgba", torch.float32)
    _require_cuda(out_depth, "out_depth", torch.float32)
    if tuple(out_rgba.shape) != (H, W, 4) or tuple(out_depth.shape) != (H, W):
        raise ValueError(f"out_rgba must be [{H}, {W}, 4] and out_depth [{H}, {W}]")
    v = _lib.splat_volume()
    v.data, v.n, v.box_lo, v.box_size = volume.data_ptr(), n, float(box_lo), float(box_size)
    o = _lib.splat_march_opts()
    o.step, o.alpha_scale, o.depth_alpha, o.stop_alpha = float(step), float(alpha_scale), float(depth_alpha), \
        float(stop_alpha)
    o.interval_lo, o.interval_hi = float(interval_lo), float(interval_hi)
    if with_interval and out_interval is None:
        out_interval = torch.empty((H, W, 2), dtype=torch.float32, device=volume.device)
    if out_interval is not None:
        _require_cuda(out_interval, "out_interval", torch.float32)
        if tuple(out_interval.shape) != (H, W, 2):
            raise ValueError(f"out_interval must be [{H}, {W}, 2]")
    c = _lib.camera_struct(cam)
    _lib.check(_lib.load().splat_raymarch(ctypes.byref(v), ctypes.byref(c), ctypes.byref(o), _ptr(out_rgba),
                                          _ptr(out_depth), _ptr(out_interval), _stream()))
    if with_interval or out_interval is not None:
        return out_rgba, out_depth, out_interval
    return out_rgba, out_depth


def _codec(box_lo, box_size: float, r_unit: float) -> _lib.splat_codec:
    c = _lib.splat_codec()
    lo = [float(box_lo)] * 3 if isinstance(box_lo, (int, float)) else [float(v) for v in box_lo]
    c.box_lo[:] = lo
    c.box_size, c.r_unit = float(box_size), float(r_unit)
    return c


def encode_samples(sph: Spheres, box_lo, box_size: float, r_unit: float):
    """Wire format of a sphere set (splat_encode_samples): (uint64-as-int64 [capacity] position+radius
    words, int32 [capacity] RGBA8 words); the first sph.count entries are valid."""
    dev = sph.centre_radius.device
    pos = torch.empty((sph.capacity,), dtype=torch.int64, device=dev)
    col = torch.empty((sph.capacity,), dtype=torch.int32, device=dev)
    c, s = _codec(box_lo, box_size, r_unit), sph.struct()
    _lib.check(_lib.load().splat_encode_samples(ctypes.byref(s), ctypes.byref(c), _ptr(pos), _ptr(col), _stream()))
    return pos, col


def decode_samples(pos: torch.Tensor, col: torch.Tensor, count: torch.Tensor, box_lo, box_size: float,
                   r_unit: float, half: bool = True, out: Spheres | None = None) -> Spheres:
    """Sphere set from the wire format (splat_decode_samples); count is a device int32 [1]."""
    _require_cuda(pos, "pos", torch.int64)
    _require_cuda(col, "col", torch.int32)
    _require_cuda(count, "count", torch.int32)
    if out is None:
        out = alloc_spheres(int(pos.numel()), pos.device, half)
    c, s = _codec(box_lo, box_size, r_unit), out.struct()
    _lib.check(_lib.load().splat_decode_samples(_ptr(pos), _ptr(col), _ptr(count), ctypes.byref(c), ctypes.byref(s),
                                                _stream()))
    return out


def build_bvh_from_samples(pos: torch.Tensor, col: torch.Tensor, count: torch.Tensor, box_lo, box_size: float,
                           r_unit: float, half: bool = True, out: Spheres | None = None, bvh: BVH | None = None,
                           ws: torch.Tensor | None = None):
    """Decode wire samples into a sphere set and build its LBVH in one call (splat_build_bvh_from_samples):
    the same spheres and BVH as decode_samples followed by build_bvh.  Returns (Spheres, BVH)."""
    _require_cuda(pos, "pos", torch.int64)
    _require_cuda(col, "col", torch.int32)
    _require_cuda(count, "count", torch.int32)
    if out is None:
        out = alloc_spheres(int(pos.numel()), pos.device, half)
    if bvh is None:
        bvh = alloc_bvh(out.capacity, pos.device)
    lib = _lib.load()
    need = lib.splat_workspace_bytes(_lib.SPLAT_OP_BUILD, out.capacity, 0, 0)
    ws = _own_ws(ws, need, pos.device, "build")
    c, s, b = _codec(box_lo, box_size, r_unit), out.struct(), bvh.struct()
    _lib.check(lib.splat_build_bvh_from_samples(_ptr(pos), _ptr(col), _ptr(count), ctypes.byref(c), ctypes.byref(s),
                                                ctypes.byref(b), _ptr(ws), ws.numel(), _stream()))
    return out, bvh


def accumulate(frame: Spheres, history: Spheres | None, history_age: torch.Tensor | None, box_lo, box_size: float,
               grid: int, max_age: int, out: Spheres | None = None, out_age: torch.Tensor | None = None,
               ws: torch.Tensor | None = None):
    """Temporal accumulation (splat_accumulate): the new frame's samples, then the history samples whose grid
    cell the frame leaves free and whose age + 1 <= max_age.  Returns (merged Spheres, uint8 ages)."""
    dev = frame.centre_radius.device
    if history is not None:
        _require_cuda(history_age, "history_age", torch.uint8)
    if out is None:
        cap = frame.capacity + (history.capacity if history is not None else 0)
        out = alloc_spheres(cap, dev, frame.half)
        if frame.src_index is None or (history is not None and history.src_index is None):
            out.src_index = None
    if out_age is None:
        out_age = torch.empty((out.capacity,), dtype=torch.uint8, device=dev)
    _require_cuda(out_age, "out_age", torch.uint8)
    o = _lib.splat_accum_opts()
    lo = [float(v) for v in (box_lo if hasattr(box_lo, "__len__") else (box_lo,) * 3)]
    for k in range(3):
        o.box_lo[k] = lo[k]
    o.box_size, o.grid, o.max_age = float(box_size), int(grid), int(max_age)
    lib = _lib.load()
    hcap = history.capacity if history is not None else 0
    ws = _own_ws(ws, lib.splat_workspace_bytes(_lib.SPLAT_OP_ACCUMULATE, hcap, int(grid), 0), dev, "accumulate")
    f, r = frame.struct(), out.struct()
    h = history.struct() if history is not None else None
    _lib.check(lib.splat_accumulate(ctypes.byref(f), ctypes.byref(h) if h is not None else None,
                                    _ptr(history_age) if history is not None else None, ctypes.byref(o),
                                    ctypes.byref(r), _ptr(out_age), _ptr(ws), ws.numel(), _stream()))
    return out, out_age


def unproject(src_cam, rgba: torch.Tensor, depth: torch.Tensor, radius_scale: float = 1.0, half: bool = True,
              out: Spheres | None = None, ws: torch.Tensor | None = None) -> Spheres:
    """Eq. 1 unprojection of a premultiplied RGBA + depth image into spheres (splat_unproject)."""
    H, W = int(src_cam.height), int(src_cam.width)
    _require_cuda(rgba, "rgba", torch.float32)
    _require_cuda(depth, "depth", torch.float32)
    if tuple(rgba.shape) != (H, W, 4) or tuple(depth.shape) != (H, W):
        raise ValueError(f"rgba must be [{H}, {W}, 4] and depth [{H}, {W}]")
    if out is None:
        out = alloc_spheres(H * W, rgba.device, half)
    lib = _lib.load()
    need = lib.splat_workspace_bytes(_lib.SPLAT_OP_UNPROJECT, 0, W, H)
    ws = _own_ws(ws, need, rgba.device, "unproject")
    cam = _lib.camera_struct(src_cam)
    s = out.struct()
    _lib.check(lib.splat_unproject(ctypes.byref(cam), _ptr(rgba), _ptr(depth), float(radius_scale), ctypes.byref(s),
                                   _ptr(ws), ws.numel(), _stream()))
    return out


def unproject_policy(src_cam, rgba: torch.Tensor, depth: torch.Tensor, mode: int, radius_scale: float = 1.0,
                     opacity_floor: float = 0.05, interval_scale: float = 1.0, interval: torch.Tensor | None = None,
                     half: bool = True, out: Spheres | None = None, ws: torch.Tensor | None = None) -> Spheres:
    """Unprojection with a radius policy (splat_unproject_policy): SPLAT_RADIUS_FOOTPRINT, _OPACITY
    (r = s fp sqrt(max(A, floor))), _INTERVAL (centre at the depth interval's midpoint,
    r = max(s fp, interval_scale half-length)) or _SPHEROID (the same centre, smeared along the ray:
    r = s fp, axis the pixel ray, half-length max(r, interval_scale half-length)); the last two need
    `interval` [H, W, 2] from `raymarch`, and _SPHEROID an output set with axes."""
    H, W = int(src_cam.height), int(src_cam.width)
    _require_cuda(rgba, "rgba", torch.float32)
    _require_cuda(depth, "depth", torch.float32)
    if tuple(rgba.shape) != (H, W, 4) or tuple(depth.shape) != (H, W):
        raise ValueError(f"rgba must be [{H}, {W}, 4] and depth [{H}, {W}]")
    if interval is not None:
        _require_cuda(interval, "interval", torch.float32)
        if tuple(interval.shape) != (H, W, 2):
            raise ValueError(f"interval must be [{H}, {W}, 2]")
    if out is None:
        out = alloc_spheres(H * W, rgba.device, half, spheroids=int(mode) == _lib.SPLAT_RADIUS_SPHEROID)
    lib = _lib.load()
    ws = _own_ws(ws, lib.splat_workspace_bytes(_lib.SPLAT_OP_UNPROJECT, 0, W, H), rgba.device, "unproject")
    pol = _lib.splat_radius_policy()
    pol.mode, pol.radius_scale = int(mode), float(radius_scale)
    pol.opacity_floor, pol.interval_scale = float(opacity_floor), float(interval_scale)
    cam = _lib.camera_struct(src_cam)
    s = out.struct()
    _lib.check(lib.splat_unproject_policy(ctypes.byref(cam), _ptr(rgba), _ptr(depth), _ptr(interval),
                                          ctypes.byref(pol), ctypes.byref(s), _ptr(ws), ws.numel(), _stream()))
    return out


@dataclass
class BVH:
    mem: torch.Tensor  # uint8 [splat_bvh_bytes(capacity)]
    capacity: int

    def struct(self) -> _lib.splat_bvh:
        b = _lib.splat_bvh()
        b.mem = self.mem.data_ptr()
        b.capacity = self.capacity
        return b

    def status(self) -> int:
        """The BVH's device status word (SPLAT_STATUS_* bits) after the current stream's work."""
        b = self.struct()
        addr = _lib.load().splat_bvh_status_word(ctypes.byref(b))
        off = int(addr) - self.mem.data_ptr()
        return int(self.mem[off:off + 4].view(torch.int32).item())


def alloc_bvh(capacity: int, device) -> BVH:
    nbytes = _lib.load().splat_bvh_bytes(int(capacity))
    return BVH(torch.zeros(nbytes, dtype=torch.uint8, device=device), int(capacity))


def build_bvh(sph: Spheres, bvh: BVH | None = None, refit_only: bool = False, ws: torch.Tensor | None = None) -> BVH:
    """LBVH build (or refit of the previous hierarchy) over a sphere set (splat_build_bvh)."""
    if bvh is None:
        bvh = alloc_bvh(sph.capacity, sph.centre_radius.device)
    lib = _lib.load()
    need = lib.splat_workspace_bytes(_lib.SPLAT_OP_BUILD, sph.capacity, 0, 0)
    ws = _own_ws(ws, need, sph.centre_radius.device, "build")
    s, b = sph.struct(), bvh.struct()
    _lib.check(lib.splat_build_bvh(ctypes.byref(s), ctypes.byref(b), int(bool(refit_only)), _ptr(ws), ws.numel(),
                                   _stream()))
    return bvh


@dataclass
class TraceOptions:
    alpha_stop: float = 0.99
    t_max: float = math.inf
    mode: int = _lib.SPLAT_ALPHA_CONSTANT
    kbuf: int = 6
    tile: tuple = field(default=(8, 8))
    schedule: int = 2  # 0 super-tiles per XCD, 1 bands, 2 heaviest tiles first
    walk: int = 2  # SPLAT_WALK_LANE (0), SPLAT_WALK_PACKET (1) or SPLAT_WALK_FRUSTUM (2)
    # raw hipEvent_t handles (torch.cuda.Event.cuda_event, after a first record) recorded around the trace
    # kernel alone; (0, 0) for none
    events: tuple = field(default=(0, 0))

    def struct(self) -> _lib.splat_trace_opts:
        o = _lib.splat_trace_opts()
        o.alpha_stop = float(self.alpha_stop)
        o.t_max = float(self.t_max)
        o.mode = int(self.mode)
        o.kbuf = int(self.kbuf)
        o.tile_w, o.tile_h = int(self.tile[0]), int(self.tile[1])
        o.schedule = int(self.schedule)
        o.walk = int(self.walk)
        o.event_begin = int(self.events[0]) or None
        o.event_end = int(self.events[1]) or None
        return o


def trace(bvh: BVH, sph: Spheres, cam, opts: TraceOptions | None = None, out: torch.Tensor | None = None,
          hits: torch.Tensor | None = None, want_hits: bool = True, ws: torch.Tensor | None = None):
    """Trace and composite from `cam` (splat_trace).  Returns (rgba [H, W, 4] float32, hits [H, W] int32 or None)."""
    opts = opts or TraceOptions()
    H, W = int(cam.height), int(cam.width)
    dev = sph.centre_radius.device
    if out is None:
        out = torch.empty((H, W, 4), dtype=torch.float32, device=dev)
    if hits is None and want_hits:
        hits = torch.empty((H, W), dtype=torch.int32, device=dev)
    _require_cuda(out, "out", torch.float32)
    if tuple(out.shape) != (H, W, 4):
        raise ValueError("out must be [H, W, 4]")
    if hits is not None and (tuple(hits.shape) != (H, W) or hits.dtype != torch.int32):
        raise ValueError("hits must be int32 [H, W]")
    lib = _lib.load()
    c, o, s, b = _lib.camera_struct(cam), opts.struct(), sph.struct(), bvh.struct()
    need = lib.splat_workspace_bytes(_lib.SPLAT_OP_TRACE, 0, W, H)
    ws = _own_ws(ws, need, dev, "trace")
    _lib.check(lib.splat_trace(ctypes.byref(b), ctypes.byref(s), ctypes.byref(c), ctypes.byref(o), _ptr(out),
                               _ptr(hits), _ptr(ws), ws.numel(), _stream()))
    return out, hits


def trace_noalloc(bvh: BVH, sph: Spheres, cam, opts: TraceOptions | None = None, out: torch.Tensor | None = None,
                  hits: torch.Tensor | None = None):
    """splat_trace_noalloc: as `trace` with caller-given outputs, with no workspace (the library's static
    device scratch holds the tile order).  Returns (out, hits)."""
    opts = opts or TraceOptions()
    H, W = int(cam.height), int(cam.width)
    _require_cuda(out, "out", torch.float32)
    if tuple(out.shape) != (H, W, 4):
        raise ValueError("out must be [H, W, 4]")
    if hits is not None and (tuple(hits.shape) != (H, W) or hits.dtype != torch.int32 or not hits.is_cuda):
        raise ValueError("hits must be int32 [H, W] on the GPU")
    lib = _lib.load()
    c, o, s, b = _lib.camera_struct(cam), opts.struct(), sph.struct(), bvh.struct()
    _lib.check(lib.splat_trace_noalloc(ctypes.byref(b), ctypes.byref(s), ctypes.byref(c), ctypes.byref(o),
                                       _ptr(out), _ptr(hits), _stream()))
    return out, hits


def alloc_grads(capacity: int, device) -> dict:
    """Zeroed per-sphere gradients: rgb [cap, 3], alpha [cap], radius [cap], centre [cap, 3], as views of one
    buffer, so that `zero_grads` clears them with one fill."""
    flat = torch.zeros((8 * capacity,), dtype=torch.float32, device=device)
    return {"rgb": flat[:3 * capacity].view(capacity, 3), "alpha": flat[3 * capacity:4 * capacity],
            "radius": flat[4 * capacity:5 * capacity], "centre": flat[5 * capacity:].view(capacity, 3)}


def zero_grads(grads: dict) -> None:
    """Clear gradients for the next accumulation: one fill when they are the views of one buffer that
    alloc_grads makes, else one fill each."""
    rgb = grads["rgb"]
    n = sum(g.numel() for g in grads.values())
    base = rgb.untyped_storage()
    shared = all(g.untyped_storage().data_ptr() == base.data_ptr() for g in grads.values())
    if shared and rgb.storage_offset() == 0 and base.nbytes() == 4 * n:
        rgb.as_strided((n,), (1,), 0).zero_()
    else:
        for g in grads.values():
            g.zero_()


def trace_backward(bvh: BVH, sph: Spheres, cam, opts: TraceOptions, out_rgba: torch.Tensor, grad_rgba: torch.Tensor,
                   grads: dict | None = None, ws: torch.Tensor | None = None) -> dict:
    """Accumulate dL/d(rgb, alpha, radius, centre) per sphere (splat_trace_backward)."""
    dev = sph.centre_radius.device
    cap = sph.capacity
    if grads is None:
        grads = alloc_grads(cap, dev)
    _require_cuda(out_rgba, "out_rgba", torch.float32)
    _require_cuda(grad_rgba, "grad_rgba", torch.float32)
    H, W = int(cam.height), int(cam.width)
    if tuple(out_rgba.shape) != (H, W, 4) or tuple(grad_rgba.shape) != (H, W, 4):
        raise ValueError("out_rgba and grad_rgba must be [H, W, 4]")
    g = _lib.splat_grads()
    g.d_rgb, g.d_alpha = grads["rgb"].data_ptr(), grads["alpha"].data_ptr()
    g.d_radius, g.d_centre = grads["radius"].data_ptr(), grads["centre"].data_ptr()
    lib = _lib.load()
    c, o, s, b = _lib.camera_struct(cam), opts.struct(), sph.struct(), bvh.struct()
    need = lib.splat_workspace_bytes(_lib.SPLAT_OP_BACKWARD, 0, W, H)
    ws = _own_ws(ws, need, dev, "trace")
    _lib.check(lib.splat_trace_backward(ctypes.byref(b), ctypes.byref(s), ctypes.byref(c), ctypes.byref(o),
                                        _ptr(out_rgba), _ptr(grad_rgba), ctypes.byref(g), _ptr(ws), ws.numel(),
                                        _stream()))
    return grads


def render(rgba: torch.Tensor, depth: torch.Tensor, src_cam, dst_cam, radius_scale: float = 1.0,
           half: bool = True, opts: TraceOptions | None = None):
    """Whole client path: unproject -> build -> trace.  Returns (image, hits, spheres, bvh)."""
    sph = unproject(src_cam, rgba, depth, radius_scale, half)
    bvh = build_bvh(sph)
    img, hits = trace(bvh, sph, dst_cam, opts)
    return img, hits, sph, bvh
