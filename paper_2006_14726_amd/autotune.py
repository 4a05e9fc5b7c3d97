"""Autotuner for the trace schedule: hits per pass (kbuf), tile shape, the
tile -> XCD schedule, the walk (per lane or per packet) and, for the batched
launch, resident waves.

Every candidate produces the same image (the traversal result does not
depend on these knobs), so the tuner only times them, with events on the
current stream, and keeps the fastest.  Results are cached in a JSON file
keyed by device architecture and a size signature of the workload.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import replace

import torch

from . import _lib
from .render import BVH, Spheres, TraceOptions, trace

TRACE_CANDIDATES = [(k, tile, sched, walk) for k in (6, 8) for tile in ((8, 8), (16, 4)) for sched in (0, 2)
                    for walk in (0, 1)]
WAVES_PER_CU = (8, 16, 32)


def cache_path() -> str:
    return os.environ.get("SPLAT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2006_14726_amd", "autotune.json"))


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: dict) -> None:
    c = _load_cache()
    c[key] = value
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _arch(device) -> str:
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def _bucket(x: int) -> int:
    return int(round(math.log2(max(int(x), 1))))


def _time(fn, reps: int) -> float:
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_trace(bvh: BVH, sph: Spheres, cam, base: TraceOptions | None = None, reps: int = 5,
               use_cache: bool = True) -> tuple[TraceOptions, dict]:
    """Fastest (kbuf, tile, schedule, walk) for tracing this sphere set from this camera size."""
    base = base or TraceOptions()
    dev = sph.centre_radius.device
    key = f"{_arch(dev)}|trace|rays{_bucket(cam.width * cam.height)}|sph{_bucket(sph.capacity)}|mode{base.mode}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            return replace(base, kbuf=hit["kbuf"], tile=tuple(hit["tile"]), schedule=hit["schedule"],
                           walk=hit.get("walk", 0)), hit
    out = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device=dev)
    hits = torch.empty((cam.height, cam.width), dtype=torch.int32, device=dev)
    timings = {}
    for k, tile, sched, walk in TRACE_CANDIDATES:
        o = replace(base, kbuf=k, tile=tile, schedule=sched, walk=walk)
        timings[f"k{k}_{tile[0]}x{tile[1]}_s{sched}_w{walk}"] = _time(
            lambda: trace(bvh, sph, cam, o, out=out, hits=hits), reps)
    best = min(timings, key=timings.get)
    k, tile, sched, walk = TRACE_CANDIDATES[list(timings).index(best)]
    rec = {"kbuf": k, "tile": list(tile), "schedule": sched, "walk": walk, "ms": timings[best], "all_ms": timings}
    _store(key, rec)
    return replace(base, kbuf=k, tile=tile, schedule=sched, walk=walk), rec


def tune_batched(renderer, reps: int = 3, use_cache: bool = True) -> dict:
    """Fastest (kbuf, tile, walk, resident waves or one grid) for a batched renderer; applies it to the renderer."""
    dev = renderer.device
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    key = f"{_arch(dev)}|batched|jobs{_bucket(renderer.n_jobs)}|rays{_bucket(renderer.rays)}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            _apply(renderer, hit)
            return hit
    renderer.prepare()
    timings = {}
    for k in (6, 8):
        for tile in ((8, 8), (16, 4)):
            for walk in (0, 1, 2):
                # persistent waves per CU, or one workgroup per (job, tile)
                for wpc in WAVES_PER_CU + (None,):
                    waves = wpc * cus if wpc else _lib.SPLAT_BATCH_GRID
                    rec = {"kbuf": k, "tile": list(tile), "walk": walk, "waves": waves}
                    _apply(renderer, rec)
                    timings[json.dumps(rec)] = _time(renderer.trace_batched, reps)
    best = min(timings, key=timings.get)
    rec = json.loads(best)
    rec["ms"] = timings[best]
    _apply(renderer, rec)
    _store(key, rec)
    return rec


def _apply(renderer, rec: dict) -> None:
    renderer.set_schedule(replace(renderer.opts, kbuf=rec["kbuf"], tile=tuple(rec["tile"]), walk=rec.get("walk", 0)),
                          rec["waves"])
