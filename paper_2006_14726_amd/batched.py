"""Many client frames, each with several target views, in one trace launch.

Every frame is unprojected and its LBVH built with the plain entry points,
the frames spread over a few streams (build lanes) so that the small frames'
builds, each a chain of short dependent kernels, run side by side; then every
(frame, view) job is traced by ONE splat_trace_batched launch:
persistent waves that pull tiles from an atomic counter until the batch is
drained, or (waves = GRID) one workgroup per (job, tile).
The whole sequence can be captured once in a HIP graph and replayed.
Outputs equal the per-job splat_trace outputs bit for bit.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import SPLAT_BATCH_GRID as GRID
from .render import (BVH, Spheres, TraceOptions, _ptr, _stream, alloc_bvh, alloc_spheres, build_bvh, trace,
                     unproject)


@dataclass
class Frame:
    rgba: torch.Tensor      # premultiplied float32 [H, W, 4] on the device
    depth: torch.Tensor     # float32 [H, W]
    src_cam: object
    dst_cams: list


class BatchedRenderer:
    """Owns the device buffers of a batch; `run()` enqueues the whole batch."""

    def __init__(self, frames: list[Frame], radius_scale: float = 1.0, half: bool = True,
                 opts: TraceOptions | None = None, waves: int = 0, build_streams: int = 4):
        self.frames = frames
        self.radius_scale = float(radius_scale)
        self.half = half
        self.opts = opts or TraceOptions()
        self.waves = int(waves)
        dev = frames[0].rgba.device
        self.device = dev
        lib = _lib.load()
        self.spheres: list[Spheres] = []
        self.bvhs: list[BVH] = []
        self.outputs: list[list[tuple[torch.Tensor, torch.Tensor]]] = []
        for fr in frames:
            cap = int(fr.src_cam.width) * int(fr.src_cam.height)
            s = alloc_spheres(cap, dev, half)
            self.spheres.append(s)
            self.bvhs.append(alloc_bvh(cap, dev))
            outs = []
            for cam in fr.dst_cams:
                outs.append((torch.zeros((cam.height, cam.width, 4), dtype=torch.float32, device=dev),
                             torch.zeros((cam.height, cam.width), dtype=torch.int32, device=dev)))
            self.outputs.append(outs)
        self._build_jobs()
        self.ws = torch.zeros(lib.splat_workspace_bytes(_lib.SPLAT_OP_BATCHED, self.n_jobs, 0, 0), dtype=torch.uint8,
                              device=dev)
        # workspaces of its own, sized for the largest frame: a captured graph
        # keeps their addresses, so no other caller may replace or free them
        # Build lanes: frames assigned largest first to the least loaded lane
        # (by source pixels); each lane has a stream and unproject and build
        # workspaces of its own, sized for its largest frame.
        n_lanes = max(1, min(int(build_streams), len(frames)))
        self.lanes: list[list[int]] = [[] for _ in range(n_lanes)]
        load = [0] * n_lanes
        for fi in sorted(range(len(frames)), key=lambda i: -self.spheres[i].capacity):
            lane = min(range(n_lanes), key=lambda k: (load[k], k))
            self.lanes[lane].append(fi)
            load[lane] += self.spheres[fi].capacity
        self.streams = [torch.cuda.Stream(device=dev) for _ in range(n_lanes)] if n_lanes > 1 else []
        self.ws_unproject, self.ws_build = [], []
        for idxs in self.lanes:
            self.ws_unproject.append(torch.empty(max(256, *(lib.splat_workspace_bytes(
                _lib.SPLAT_OP_UNPROJECT, 0, frames[i].src_cam.width, frames[i].src_cam.height) for i in idxs)),
                dtype=torch.uint8, device=dev))
            self.ws_build.append(torch.empty(max(256, *(lib.splat_workspace_bytes(
                _lib.SPLAT_OP_BUILD, self.spheres[i].capacity, 0, 0) for i in idxs)), dtype=torch.uint8, device=dev))
        # buffers written on a lane stream are not reused by the allocator
        # before that stream's work at their release has finished
        for lane, st in enumerate(self.streams):
            for t in (self.ws_unproject[lane], self.ws_build[lane]):
                t.record_stream(st)
            for fi in self.lanes[lane]:
                s = self.spheres[fi]
                for t in (s.centre_radius, s.rgba, s.count, s.src_index, s.axis, self.bvhs[fi].mem):
                    if t is not None:
                        t.record_stream(st)
        self.ws_trace = torch.empty(max(256, *(lib.splat_workspace_bytes(_lib.SPLAT_OP_TRACE, 0, c.width, c.height)
                                                 for fr in frames for c in fr.dst_cams)), dtype=torch.uint8, device=dev)
        self.graph = None

    def set_schedule(self, opts: TraceOptions, waves: int) -> None:
        """Change hits per pass, tile shape or resident waves (rebuilds the tile prefix)."""
        self.opts = opts
        self.waves = int(waves)
        self._build_jobs()
        self.graph = None

    def _build_jobs(self) -> None:
        """Job table and exclusive tile prefix, built on the host and copied once."""
        frames, half, dev = self.frames, self.half, self.device
        tw, th = self.opts.tile
        jobs, offsets, total = [], [0], 0
        for fi, fr in enumerate(frames):
            for vi, cam in enumerate(fr.dst_cams):
                j = _lib.splat_batch_job()
                j.bvh_mem = self.bvhs[fi].mem.data_ptr()
                j.bvh_capacity = self.bvhs[fi].capacity
                j.centre_radius = self.spheres[fi].centre_radius.data_ptr()
                j.rgba = self.spheres[fi].rgba.data_ptr()
                j.rgba_dtype = _lib.SPLAT_F16 if half else _lib.SPLAT_F32
                j.camera = _lib.camera_struct(cam)
                j.out_rgba = self.outputs[fi][vi][0].data_ptr()
                j.out_hits = self.outputs[fi][vi][1].data_ptr()
                jobs.append(j)
                total += ((cam.width + tw - 1) // tw) * ((cam.height + th - 1) // th)
                offsets.append(total)
        self.n_jobs = len(jobs)
        self.total_tiles = total
        self.rays = sum(int(c.width) * int(c.height) for fr in frames for c in fr.dst_cams)
        table = (_lib.splat_batch_job * self.n_jobs)(*jobs)
        raw = np.frombuffer(bytes(table), dtype=np.uint8)
        self.job_table = torch.from_numpy(raw.copy()).to(dev)
        self.tile_offsets = torch.tensor(np.array(offsets[:-1], dtype=np.uint32).view(np.int32), device=dev)

    def _prepare_lane(self, lane: int) -> None:
        for fi in self.lanes[lane]:
            fr, s = self.frames[fi], self.spheres[fi]
            unproject(fr.src_cam, fr.rgba, fr.depth, self.radius_scale, self.half, out=s, ws=self.ws_unproject[lane])
            build_bvh(s, self.bvhs[fi], ws=self.ws_build[lane])

    def prepare(self):
        """Unproject and build every frame (plain launches).  With several
        lanes each lane's stream waits for the work already on the current
        stream, and the current stream waits for every lane: under capture
        the lanes become parallel branches of the graph."""
        if not self.streams:
            self._prepare_lane(0)
            return
        cur = torch.cuda.current_stream(self.device)
        for lane, st in enumerate(self.streams):
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                self._prepare_lane(lane)
        for st in self.streams:
            cur.wait_stream(st)

    def trace_batched(self):
        """Every job in one persistent launch (splat_trace_batched)."""
        o = self.opts.struct()
        _lib.check(_lib.load().splat_trace_batched(_ptr(self.job_table), _ptr(self.tile_offsets), self.n_jobs,
                                                   self.total_tiles, ctypes.byref(o), self.waves, _ptr(self.ws),
                                                   self.ws.numel(), _stream()))

    def run(self):
        self.prepare()
        self.trace_batched()

    def run_sequential(self):
        """Reference schedule: the same work as plain per-job launches."""
        self.prepare()
        for fi, fr in enumerate(self.frames):
            for vi, cam in enumerate(fr.dst_cams):
                out, hits = self.outputs[fi][vi]
                trace(self.bvhs[fi], self.spheres[fi], cam, self.opts, out=out, hits=hits, ws=self.ws_trace)

    def capture(self):
        """Capture run() into a HIP graph (torch.cuda.CUDAGraph over hipGraph)."""
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run()  # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
