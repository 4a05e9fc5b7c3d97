"""Benchmark of the client-side splat path on one MI355X.

One step = unproject (Eq. 1) -> LBVH build -> trace + composite of the
1024^2 -> 1920x1080 client frame (64 blobs, 256^3 volume, 10 deg yaw + 3 deg
pitch, radius = 1 footprint, half colours), with the source image already in
HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps 20] [--warmup 5] [--scale 1.0] [--no-cpu]
"""
from __future__ import annotations

import argparse
import copy
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--scale", type=float, default=1.0)
    p.add_argument("--kbuf", type=int, default=6)
    p.add_argument("--tile", type=str, default="8x8")
    p.add_argument("--walk", type=int, default=2, help="0 per-lane BVH walk, 1 packet walk, 2 frustum walk")
    p.add_argument("--schedule", type=int, default=2, help="tile order: 0 super-tiles per XCD, 1 bands, 2 heaviest first")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-bwd", action="store_true", help="skip the fwd+bwd measurement")
    p.add_argument("--batch-frames", type=int, default=64,
                   help="frames of the batched graph measurement (0 skips it)")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the radius-scale sweep, the large-frame orbit and the copy bandwidth")
    p.add_argument("--orbit-frames", type=int, default=30, help="frames of the large-frame orbit (0 skips it)")
    p.add_argument("--workload", choices=("client", "large"), default="client",
                   help="client: 1024^2 source -> 1920x1080 (the headline); large: 3840x2160 -> 3840x2160 at yaw 15 "
                        "(for the counter report of the large frame)")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="run one plain device copy of this many MiB first (scales the HBM byte counters)")
    return p.parse_args()


def source_hash(files) -> str:
    """sha256[:16] of kernel sources, as recorded in the profile summaries they were measured from."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2006_14726_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRACE_SOURCES = ("trace.hip", "common.h", "kernels.h")
BUILD_SOURCES = ("bvh.hip", "common.h", "kernels.h")


def profile_record(name: str, args, sources=TRACE_SOURCES, key="trace_source_sha256_16"):
    """key = value lines of a committed profile summary, or None when the file is missing, the kernel
    sources differ from the ones profiled or the launch configuration is not the profiled one."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path) or (args.kbuf, args.tile, args.scale, args.walk, args.schedule) != (6, "8x8", 1.0, 2, 2):
        return None
    rec = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            rec[k.strip()] = v.strip()
    if rec.get(key) != source_hash(sources):
        return None
    return rec


def measured_traffic(args, workload="client_frame"):
    """HBM bytes per trace launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None."""
    rec = profile_record(f"trace_{workload}_hbm_traffic.txt", args)
    return None if rec is None else int(float(rec["traffic_bytes_per_dispatch"]))


def l2_hit_rate(args, workload="client_frame"):
    """L2 (TCC) hit rate of the trace kernel from the committed TCC_HIT/TCC_MISS summary, or None."""
    rec = profile_record(f"trace_{workload}_l2.txt", args)
    return None if rec is None else float(rec["l2_hit_rate"])


def valu_issue(args, kernel_ms: float, workload="client_frame"):
    """Vector-issue occupancy of the trace kernel from the committed SQ counter summary: wave64 vector
    instructions x 4 cycles / 1024 SIMDs, over the kernel's duration at 2.4 GHz; None when the kernel
    source or the launch configuration differs from the one profiled."""
    rec = profile_record(f"trace_{workload}_sq_counters.txt", args)
    if rec is None:
        return None
    valu = float(rec["sq_insts_valu_per_dispatch"])
    busy = valu * 4 / 1024 / (kernel_ms * 1e-3 * 2.4e9)
    return {"valu_insts_per_launch": int(valu), "valu_insts_per_wave": float(rec["sq_insts_valu_per_wave"]),
            "valu_busy_frac": round(busy, 3),
            "note": "vector-instruction issue: the bound of this kernel (4 cycles per wave64 instruction, 1024 SIMDs, 2.4 GHz)"}


# Build bytes per sphere as implemented (30-bit codes, four 8-bit radix passes):
#   bounds 16 (centres) + Morton 24 (centres in, key and id out) + sort 4 x 16 (key and id in and out)
#   + 12 (three digit histograms read the keys) + Karras 44 (sorted key and id in; per node two
#   references and the axis, parent, key range and arrival flag; per leaf its parent and id)
#   + refit 92 (centre, radius and colour word in, leaf id and parent, node parent and range; 48 B
#   of child slots out)
# and per internal node the 4-wide node: 3 x 64 B of binary nodes in, 128 B out.
BUILD_BYTES_PER_SPHERE = 16 + 24 + 4 * 16 + 12 + 44 + 92
BUILD_BYTES_PER_NODE = 3 * 64 + 128


def build_bytes(n: int) -> int:
    return n * BUILD_BYTES_PER_SPHERE + max(n - 1, 0) * BUILD_BYTES_PER_NODE


def trace_bytes(n: int, pixels: int, half: bool) -> int:
    """Compulsory bytes of one trace: sphere geometry + colour, hierarchy, output image and hit counts."""
    cb = 8 if half else 16
    return n * (16 + cb) + max(n - 1, 0) * 56 + pixels * (16 + 4)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2006_14726_amd as sp
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.calib_copy_mib > 0:
        n_words = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n_words, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    work = synth.CLIENT_FRAME if args.workload == "client" else synth.LARGE
    rgba_np, depth_np, src, dst = synth.source_image(work)
    rgba = torch.from_numpy(rgba_np).to(dev)
    depth = torch.from_numpy(depth_np).to(dev)
    tw, th = (int(v) for v in args.tile.split("x"))
    opts = sp.TraceOptions(alpha_stop=0.99, kbuf=args.kbuf, tile=(tw, th), walk=args.walk, schedule=args.schedule)
    P = dst.width * dst.height

    sph = sp.alloc_spheres(src.width * src.height, dev, half=True)
    bvh = sp.alloc_bvh(sph.capacity, dev)
    out = torch.empty((dst.height, dst.width, 4), dtype=torch.float32, device=dev)
    hits = torch.empty((dst.height, dst.width), dtype=torch.int32, device=dev)

    def step(ev=None):
        if ev: ev[0].record()
        sp.unproject(src, rgba, depth, args.scale, True, out=sph)
        if ev: ev[1].record()
        sp.build_bvh(sph, bvh)
        if ev: ev[2].record()
        sp.trace(bvh, sph, dst, opts, out=out, hits=hits)
        if ev: ev[3].record()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # whole-step wall clock
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps

    # the same step captured once in a HIP graph and replayed (one host
    # submission per step instead of the three calls' launches); its image
    # must equal the eager step's bit for bit
    eager_img, eager_hits = out.clone(), hits.clone()
    step_graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(step_graph):
        step()
    out.fill_(-1.0)
    hits.fill_(-1)
    step_graph.replay()
    torch.cuda.synchronize()
    graph_same = bool(torch.equal(out, eager_img) and torch.equal(hits, eager_hits))
    for _ in range(args.warmup):
        step_graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_graph.replay()
    torch.cuda.synchronize()
    graph_wall = (time.perf_counter() - t0) / args.steps
    del eager_img, eager_hits

    # per-stage device time (events on the stream the kernels are launched on)
    stage = np.zeros((args.steps, 3))
    for i in range(args.steps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        step(ev)
        torch.cuda.synchronize()
        stage[i] = [ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2]), ev[2].elapsed_time(ev[3])]
    n = sph.n()

    # trace kernel alone, back to back
    reps = max(args.steps, 10)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sp.trace(bvh, sph, dst, opts, out=out, hits=hits)
    e1.record()
    torch.cuda.synchronize()
    call_ms = e0.elapsed_time(e1) / reps
    # the trace kernel alone: the library records a pair of events right
    # around it (after the tile ordering), one pair per launch, back to back
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in pairs:  # a first record creates the underlying events
        a.record()
        b.record()
    torch.cuda.synchronize()
    for a, b in pairs:
        o_ev = copy.copy(opts)
        o_ev.events = (a.cuda_event, b.cuda_event)
        sp.trace(bvh, sph, dst, o_ev, out=out, hits=hits)
    torch.cuda.synchronize()
    trace_ms = float(np.mean([a.elapsed_time(b) for a, b in pairs]))
    tb = trace_bytes(n, P, True)
    achieved = tb / (trace_ms * 1e-3) / 1e9
    wl = "client_frame" if args.workload == "client" else "large_frame"
    build_ms = float(np.median(stage[:, 1]))
    bb = build_bytes(n)

    # cold: L2 and MALL flushed by writing a 512 MiB buffer before each trace
    flush = torch.empty(1 << 27, dtype=torch.float32, device=dev)
    cold = []
    for _ in range(5):
        flush.fill_(1.0)
        cold.append(_events(torch, [lambda: sp.trace(bvh, sph, dst, opts, out=out, hits=hits)])[0])
    del flush

    hit_stats = hits.float()
    result = {
        "metric": "Mrays/s trace+composite (whole unproject+build+trace step), fwd+bwd ms vs fwd-only, "
                  "at <=1e-4 RGBA err",
        "value": round(P / wall / 1e6, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 ray/sphere tests, f32 boxes+compositing, f16 colours",
        "data": "synthetic seeded blob volume, CPU ray-cast 2.5D source image",
        "config": {"workload": f"{'client' if args.workload == 'client' else 'large'} frame: {src.width}x{src.height} "
                               f"source ({n} spheres, radius scale {args.scale}) -> {dst.width}x{dst.height} target, "
                               f"yaw {work.yaw} pitch {work.pitch}",
                   "rays": P, "spheres": n, "kbuf": args.kbuf, "tile": args.tile,
                   "walk": ["per-lane", "packet", "frustum"][args.walk],
                   "schedule": ["xcd super-tiles", "xcd bands", "heaviest first"][args.schedule], "alpha_stop": 0.99},
        "stages_ms": {"unproject": round(float(np.median(stage[:, 0])), 4),
                      "build": round(float(np.median(stage[:, 1])), 4),
                      "trace": round(float(np.median(stage[:, 2])), 4)},
        "stages_p10_p90_ms": {k: [round(float(np.percentile(stage[:, i], 10)), 4),
                                  round(float(np.percentile(stage[:, i], 90)), 4)]
                              for i, k in enumerate(("unproject", "build", "trace"))},
        "graph_step": {"ms_per_step": round(graph_wall * 1e3, 4), "mrays_s": round(P / graph_wall / 1e6, 3),
                       "bit_identical": graph_same},
        "trace_only_mrays_s": round(P / (call_ms * 1e-3) / 1e6, 2),
        "trace_call_ms": round(call_ms, 4),
        "trace_cold_ms": round(float(np.median(cold)), 4),
        "mean_hits_per_ray": round(float(hit_stats.mean()), 3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": measured_traffic(args, wl),
                     "kernel": f"k_trace<{args.kbuf}, false, {args.walk}>",
                     "algorithmic_bytes": tb, "avg_launch_ms": round(trace_ms, 4),
                     "l2_hit_rate": l2_hit_rate(args, wl),
                     "note": "avg_launch_ms is the trace kernel alone, between events the library records around "
                             "it; trace_call_ms adds the tile-ordering kernels of schedule 2",
                     "issue": valu_issue(args, trace_ms, wl)},
        "build_roofline": {"bound": "hbm", "achieved": round(bb / (build_ms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(bb / (build_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                           "algorithmic_bytes": bb, "build_ms": round(build_ms, 4),
                           "bytes_per_sphere": BUILD_BYTES_PER_SPHERE, "bytes_per_internal_node": BUILD_BYTES_PER_NODE,
                           "note": "the whole splat_build_bvh call (every build kernel) between events; bytes as "
                                   "implemented: four 8-bit radix passes and the 4-wide node gather"},
    }
    result["l2_hit_rate"] = result["roofline"]["l2_hit_rate"]

    if not args.no_extra:
        result["copy_gbs"] = copy_bandwidth(torch, dev)
        result["roofline"]["frac_of_copy"] = round(achieved / result["copy_gbs"], 5)
        result["scale_sweep"] = scale_sweep(sp, torch, src, rgba, depth, dst, opts, max(args.steps, 20))
        if args.orbit_frames > 0:
            result["large_orbit"] = large_orbit(sp, torch, synth, dev, opts, args.orbit_frames, args)
        result["server_stage"] = server_stage(sp, torch, synth, dev, src, dst, opts, max(args.steps, 10))
        result["codec"] = codec(sp, torch, synth, sph, bvh, src, dst, opts, max(args.steps, 10))
        result["accumulate"] = accumulate(sp, torch, synth, dev, src, sph, max(args.steps, 10))
        result["radius_policies"] = radius_policies(sp, torch, synth, dev, src, dst, opts, max(args.steps, 10))
    if not args.no_bwd:
        result["fwd_bwd"] = fwd_bwd(sp, torch, synth, dev, args.steps)
    if args.batch_frames > 0:
        result["batched"] = batched(sp, torch, synth, dev, args.batch_frames)
    if not args.no_cpu:
        result["cpu_baseline"], orc = cpu_baseline(rgba_np, depth_np, src, dst, args.scale)
        result["parity"] = parity(sp, torch, dev, orc, sph, dst, opts)
    print(json.dumps(result), flush=True)


def _compare(g, n, orc, tol=1e-4):
    """GPU pixels against the oracle's (same rules as the parity tests): a pixel passes within `tol` per
    channel with the same composited hit count, on the oracle's main result or, at a knife-edge, on its
    alternate; a pixel where a sphere grazes the ray (or with two knife-edges) is exempt."""
    import oracle
    g = np.asarray(g, dtype=np.float64).reshape(-1, 4)
    n = np.asarray(n).reshape(-1).astype(np.int64)
    flags = orc["flags"]
    exempt = (flags & (oracle.FLAG_GRAZE | oracle.FLAG_MULTI_KNIFE)) != 0
    err = np.abs(g - orc["rgba"]).max(axis=1)
    err_alt = np.abs(g - orc["alt_rgba"]).max(axis=1)
    ok_alt = (err_alt <= tol) & (n == orc["alt_n"]) & ((flags & oracle.FLAG_KNIFE) != 0)
    ok = ((err <= tol) & (n == orc["n"])) | ok_alt | exempt
    strict = ~exempt
    e = np.where(strict, np.where(ok_alt, np.minimum(err, err_alt), err), 0.0)
    return {"pixels": int(g.shape[0]), "max_err": float(e.max()) if e.size else 0.0,
            "mismatches": int((~ok).sum()), "exempt": int(exempt.sum()),
            "knife": int(((flags & oracle.FLAG_KNIFE) != 0).sum()), "hits_checked": int(n[strict].sum())}


def parity(sp, torch, dev, orc, sph, dst, opts):
    """The timed configuration against the FP64 oracle, on the pixels the CPU baseline rendered.
    Unprojection: the timed GPU sphere set against the oracle's own unprojection of the same image
    (count and order exact, centre and radius within 1 ulp, colours bit-exact).  Trace: the oracle's
    sphere set uploaded, built and traced with the timed options, compared pixel by pixel (<= 1e-4 per
    RGBA channel, exact hit counts; grazing pixels exempt up to 1e-4 of the pixels)."""
    cr, col, idx = orc["spheres"]
    n = sph.n()
    g_cr = sph.centre_radius[:n].cpu().numpy()
    unp = {"count_equal": bool(n == cr.shape[0])}
    if unp["count_equal"]:
        unp["order_equal"] = bool(np.array_equal(sph.src_index[:n].cpu().numpy().view(np.uint32), idx))
        unp["max_ulp"] = int(np.abs(g_cr.view(np.int32).astype(np.int64) - cr.view(np.int32)).max())
        unp["colours_equal"] = bool(np.array_equal(sph.rgba[:n].cpu().numpy().view(np.uint16), col.view(np.uint16)))
    s2 = sp.spheres_from_tensors(torch.from_numpy(cr).to(dev), torch.from_numpy(col).to(dev))
    img, hits = sp.trace(sp.build_bvh(s2), s2, dst, opts)
    torch.cuda.synchronize()
    pix = orc["pixels"]
    st = _compare(img.cpu().numpy().reshape(-1, 4)[pix], hits.cpu().numpy().reshape(-1)[pix], orc["render"])
    st["exempt_budget"] = max(1, int(1e-4 * st["pixels"]))
    st["ok"] = bool(st["mismatches"] == 0 and st["exempt"] <= st["exempt_budget"] and unp.get("max_ulp", 9) <= 1
                    and unp.get("order_equal") and unp.get("colours_equal"))
    st["unproject"] = unp
    st["tolerance"] = "max abs 1e-4 per RGBA channel, exact hit counts, FP64 oracle on the same sphere arrays"
    return st


def fwd_bwd(sp, torch, synth, dev, steps):
    """Differentiable config: 512^2 source, soft alpha, float colours; forward vs forward+backward,
    both with the trace schedule the autotuner picks for this workload's forward."""
    from paper_2006_14726_amd import autotune
    rgba_np, depth_np, src, dst = synth.source_image(synth.DIFF)
    s = sp.unproject(src, torch.from_numpy(rgba_np).to(dev), torch.from_numpy(depth_np).to(dev), 1.0, False)
    bvh = sp.build_bvh(s)
    opts, _ = autotune.tune_trace(bvh, s, dst, sp.TraceOptions(mode=sp.SPLAT_ALPHA_SOFT), use_cache=False)
    out, _ = sp.trace(bvh, s, dst, opts, want_hits=False)
    grad = torch.randn_like(out)
    grads = sp.trace_backward(bvh, s, dst, opts, out, grad)
    torch.cuda.synchronize()
    reps = max(steps, 10)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        sp.trace(bvh, s, dst, opts, out=out, want_hits=False)
    ev[1].record()
    for _ in range(reps):
        sp.zero_grads(grads)
        sp.trace(bvh, s, dst, opts, out=out, want_hits=False)
        sp.trace_backward(bvh, s, dst, opts, out, grad, grads)
    ev[2].record()
    torch.cuda.synchronize()
    f = ev[0].elapsed_time(ev[1]) / reps
    fb = ev[1].elapsed_time(ev[2]) / reps
    return {"workload": f"{src.width}x{src.height} source ({s.n()} spheres) -> {dst.width}x{dst.height}, soft alpha",
            "fwd_ms": round(f, 4), "fwd_bwd_ms": round(fb, 4), "bwd_over_fwd": round((fb - f) / f, 3),
            "tuned": {"kbuf": opts.kbuf, "tile": list(opts.tile), "schedule": opts.schedule, "walk": opts.walk}}


def batched(sp, torch, synth, dev, n_frames):
    """Uneven client frames (source 256^2..2048^2, target 640x480..1920x1080, 1-8 views each):
    one graph-captured persistent launch vs per-job plain launches, bit-identical outputs."""
    from paper_2006_14726_amd import autotune
    from paper_2006_14726_amd.batched import BatchedRenderer, Frame
    t0 = time.perf_counter()
    frames = []
    for fr in synth.batch_frames(n_frames):
        rgba, depth, src, dsts = synth.batch_frame_images(fr)
        frames.append(Frame(torch.from_numpy(rgba).to(dev), torch.from_numpy(depth).to(dev), src, dsts))
    gen_s = time.perf_counter() - t0
    r = BatchedRenderer(frames, half=True)
    tuned = autotune.tune_batched(r, use_cache=False)

    def wall(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps

    seq = wall(r.run_sequential)
    ref = [[o.clone() for o, _ in views] for views in r.outputs]
    r.capture()
    graph = wall(r.replay)
    same = all(torch.equal(o, q) for views, rv in zip(r.outputs, ref) for (o, _), q in zip(views, rv))
    return {"workload": f"{n_frames} frames, {r.n_jobs} views, {r.rays} rays, "
                        f"{sum(int(f.src_cam.width) * int(f.src_cam.height) for f in frames)} source pixels",
            "graph_ms": round(graph * 1e3, 3), "sequential_ms": round(seq * 1e3, 3),
            "graph_mrays_s": round(r.rays / graph / 1e6, 1), "sequential_mrays_s": round(r.rays / seq / 1e6, 1),
            "bit_identical": bool(same), "tuned": {k: tuned[k] for k in ("kbuf", "tile", "walk", "waves")},
            "build_lanes": len(r.lanes),
            "input_generation_s": round(gen_s, 1)}


def _events(torch, fns):
    """Device ms of each callable in `fns`, run back to back, events on the launch stream."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(len(fns) + 1)]
    ev[0].record()
    for i, fn in enumerate(fns):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(len(fns))]


def copy_bandwidth(torch, dev):
    """Achievable HBM bandwidth: a 1 GiB device-to-device copy (2 GiB moved), best of 5."""
    a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    best = min(_events(torch, [lambda: b.copy_(a)])[0] for _ in range(5))
    del a, b
    return round(2 * (1 << 30) / (best * 1e-3) / 1e9, 1)


def scale_sweep(sp, torch, src, rgba, depth, dst, opts, reps):
    """Client frame at radius scale 0.5, 1, 2: median, p10 and p90 of each stage."""
    out = {}
    for scale in (0.5, 1.0, 2.0):
        sph = sp.unproject(src, rgba, depth, scale, True)
        bvh = sp.build_bvh(sph)
        img, hits = sp.trace(bvh, sph, dst, opts)
        t = np.array([_events(torch, [lambda: sp.unproject(src, rgba, depth, scale, True, out=sph),
                                      lambda: sp.build_bvh(sph, bvh),
                                      lambda: sp.trace(bvh, sph, dst, opts, out=img, hits=hits)])
                      for _ in range(reps)])
        rec = {"spheres": sph.n()}
        for i, k in enumerate(("unproject", "build", "trace")):
            rec[k] = [round(float(np.percentile(t[:, i], q)), 4) for q in (50, 10, 90)]
        rec["trace_mrays_s"] = round(dst.width * dst.height / (np.median(t[:, 2]) * 1e-3) / 1e6, 1)
        out[f"s{scale}"] = rec
    out["format"] = "stage: [median, p10, p90] ms"
    return out


def large_orbit(sp, torch, synth, dev, opts, frames, args):
    """Large frame: 3840x2160 source -> 3840x2160 targets at yaw 15 + k deg, k = 0..frames-1;
    unproject, rebuild and trace every frame."""
    rgba_np, depth_np, src, dst0 = synth.source_image(synth.LARGE)
    rgba = torch.from_numpy(rgba_np).to(dev)
    depth = torch.from_numpy(depth_np).to(dev)
    sph = sp.alloc_spheres(src.width * src.height, dev, half=True)
    bvh = sp.alloc_bvh(sph.capacity, dev)
    img = torch.empty((dst0.height, dst0.width, 4), dtype=torch.float32, device=dev)
    hits = torch.empty((dst0.height, dst0.width), dtype=torch.int32, device=dev)
    cams = [synth.rotated_camera(src, synth.LARGE.yaw + k, 0.0) for k in range(frames)]
    sp.unproject(src, rgba, depth, 1.0, True, out=sph)
    sp.build_bvh(sph, bvh)
    sp.trace(bvh, sph, cams[0], opts, out=img, hits=hits)  # warm
    t = np.array([_events(torch, [lambda: sp.unproject(src, rgba, depth, 1.0, True, out=sph),
                                  lambda: sp.build_bvh(sph, bvh),
                                  lambda c=c: sp.trace(bvh, sph, c, opts, out=img, hits=hits)]) for c in cams])
    # the trace kernel alone per pose (events the library records around it)
    pairs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cams]
    for a, b in pairs:
        a.record()
        b.record()
    torch.cuda.synchronize()
    for (a, b), c in zip(pairs, cams):
        o_ev = copy.copy(opts)
        o_ev.events = (a.cuda_event, b.cuda_event)
        sp.trace(bvh, sph, c, o_ev, out=img, hits=hits)
    torch.cuda.synchronize()
    kern = np.array([a.elapsed_time(b) for a, b in pairs])
    rays = dst0.width * dst0.height
    frame = t.sum(axis=1)
    res = {"workload": f"{src.width}x{src.height} source ({sph.n()} spheres) -> {dst0.width}x{dst0.height}, "
                       f"yaw {synth.LARGE.yaw}+k deg, k = 0..{frames - 1}, rebuilt every frame",
           "frame_ms_mean": round(float(frame.mean()), 4), "frame_mrays_s": round(rays / (frame.mean() * 1e-3) / 1e6, 1),
           "trace_mrays_s": round(rays / (t[:, 2].mean() * 1e-3) / 1e6, 1)}
    for i, k in enumerate(("unproject", "build", "trace")):
        res[k + "_ms"] = [round(float(t[:, i].mean()), 4), round(float(t[:, i].min()), 4), round(float(t[:, i].max()), 4)]
    res["format"] = "stage_ms: [mean, min, max] over the frames"
    n = sph.n()
    tb = trace_bytes(n, rays, True)
    ach = tb / (float(kern.mean()) * 1e-3) / 1e9
    res["roofline"] = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(ach / HBM_PEAK_GBS, 5), "algorithmic_bytes": tb,
                       "avg_launch_ms": round(float(kern.mean()), 4), "kernel": "trace kernel alone, mean over the poses",
                       "traffic": measured_traffic(args, "large_frame"),
                       "l2_hit_rate": l2_hit_rate(args, "large_frame"),
                       "pose0_launch_ms": round(float(kern[0]), 4),
                       "issue": valu_issue(args, float(kern[0]), "large_frame"),
                       "note": "traffic, l2_hit_rate and issue are the committed counter figures of pose k = 0 "
                               "(yaw 15), the launch profiled with --workload large"}
    bb = build_bytes(n)
    bms = float(t[:, 1].mean())
    res["build_roofline"] = {"bound": "hbm", "achieved": round(bb / (bms * 1e-3) / 1e9, 2), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(bb / (bms * 1e-3) / 1e9 / HBM_PEAK_GBS, 5),
                             "algorithmic_bytes": bb, "build_ms": round(bms, 4)}
    del sph, bvh, img, hits
    return res


def server_stage(sp, torch, synth, dev, src, dst, opts, reps):
    """The stage before the path on the GPU: ray-march the client frame's 256^3 volume into the 1024^2
    source image, then the whole server + client frame (march, unproject, build, trace)."""
    vol = torch.from_numpy(synth.volume_of(synth.CLIENT_FRAME)).to(dev)
    rgba, depth = sp.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src)
    sph = sp.unproject(src, rgba, depth, 1.0, True)
    bvh = sp.build_bvh(sph)
    img, hits = sp.trace(bvh, sph, dst, opts)
    t = np.array([_events(torch, [lambda: sp.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src, out_rgba=rgba,
                                                      out_depth=depth),
                                  lambda: sp.unproject(src, rgba, depth, 1.0, True, out=sph),
                                  lambda: sp.build_bvh(sph, bvh),
                                  lambda: sp.trace(bvh, sph, dst, opts, out=img, hits=hits)]) for _ in range(reps)])
    med = np.median(t, axis=0)
    return {"workload": f"256^3 volume -> {src.width}x{src.height} source ({sph.n()} spheres) -> "
                        f"{dst.width}x{dst.height} target",
            "march_ms": round(float(med[0]), 4),
            "march_mrays_s": round(src.width * src.height / (med[0] * 1e-3) / 1e6, 1),
            "frame_ms": round(float(t.sum(axis=1).mean()), 4),
            "stages_ms": {k: round(float(v), 4) for k, v in zip(("march", "unproject", "build", "trace"), med)}}


def radius_policies(sp, torch, synth, dev, src, dst, opts, reps):
    """The client frame under each radius policy: the GPU marcher with the depth interval, then
    unproject (policy), build and trace; per policy the stage times, the mean composited hits and
    the mean image change against the footprint policy."""
    vol = torch.from_numpy(synth.volume_of(synth.CLIENT_FRAME)).to(dev)
    rgba, depth, itv = sp.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src, with_interval=True)
    out, base = {}, None
    for name, mode, kw in (("footprint", sp.SPLAT_RADIUS_FOOTPRINT, {}),
                           ("opacity", sp.SPLAT_RADIUS_OPACITY, {"opacity_floor": 0.05}),
                           ("interval", sp.SPLAT_RADIUS_INTERVAL, {"interval_scale": 0.1}),
                           ("interval_wide", sp.SPLAT_RADIUS_INTERVAL, {"interval_scale": 0.25}),
                           ("spheroid", sp.SPLAT_RADIUS_SPHEROID, {"interval_scale": 0.1}),
                           ("spheroid_wide", sp.SPLAT_RADIUS_SPHEROID, {"interval_scale": 0.25}),
                           ("spheroid_full", sp.SPLAT_RADIUS_SPHEROID, {"interval_scale": 1.0})):
        sph = sp.unproject_policy(src, rgba, depth, mode, interval=itv, **kw)
        bvh = sp.build_bvh(sph)
        img, hits = sp.trace(bvh, sph, dst, opts)
        t = np.array([_events(torch, [lambda: sp.unproject_policy(src, rgba, depth, mode, interval=itv, out=sph, **kw),
                                      lambda: sp.build_bvh(sph, bvh),
                                      lambda: sp.trace(bvh, sph, dst, opts, out=img, hits=hits)])
                      for _ in range(reps)])
        med = np.median(t, axis=0)
        # wide spheres overlap many times over: a larger hit buffer saturates the stop in fewer passes
        o16 = copy.copy(opts)
        o16.kbuf = 16
        sp.trace(bvh, sph, dst, o16, out=img, hits=hits)
        t16 = float(np.median([_events(torch, [lambda: sp.trace(bvh, sph, dst, o16, out=img, hits=hits)])[0]
                               for _ in range(reps)]))
        if base is None:
            base = img.clone()
        r = sph.centre_radius[:sph.n(), 3]
        extra = {}
        if sph.axis is not None:
            extra["median_half_length"] = round(float(sph.axis[:sph.n(), 3].median()), 6)
        out[name] = {"params": kw, "spheres": sph.n(), "median_radius": round(float(r.median()), 6), **extra,
                     "mean_hits": round(float(hits.float().mean()), 3),
                     "stages_ms": {k: round(float(v), 4) for k, v in zip(("unproject", "build", "trace"), med)},
                     "trace_ms_kbuf16": round(t16, 4),
                     "image_mean_abs_change": round(float((img - base).abs().mean()), 6)}
    foot = out["footprint"]["stages_ms"]["trace"]
    for name in out:
        out[name]["trace_over_footprint"] = round(out[name]["stages_ms"]["trace"] / foot, 3)
    return out


def codec(sp, torch, synth, sph, bvh, src, dst, opts, reps):
    """Wire format of the client frame's spheres: encode + decode time, bytes, and the image change."""
    ru = 2.0 * src.tan_half_fov_y / src.height
    pos, col = sp.encode_samples(sph, synth.BOX_LO, synth.BOX_SIZE, ru)
    dec = sp.decode_samples(pos, col, sph.count, synth.BOX_LO, synth.BOX_SIZE, ru, half=True)
    t = np.array([_events(torch, [lambda: sp.encode_samples(sph, synth.BOX_LO, synth.BOX_SIZE, ru),
                                  lambda: sp.decode_samples(pos, col, sph.count, synth.BOX_LO, synth.BOX_SIZE, ru,
                                                            half=True, out=dec)]) for _ in range(reps)])
    img, _ = sp.trace(bvh, sph, dst, opts)
    dbvh = sp.build_bvh(dec)
    dimg, _ = sp.trace(dbvh, dec, dst, opts)
    diff = (img - dimg).abs()
    n = sph.n()
    # decode then build, against the build that decodes the samples in its first kernel
    fused, fbvh = sp.build_bvh_from_samples(pos, col, sph.count, synth.BOX_LO, synth.BOX_SIZE, ru, half=True)
    tb = np.array([_events(torch, [lambda: sp.decode_samples(pos, col, sph.count, synth.BOX_LO, synth.BOX_SIZE, ru,
                                                              half=True, out=dec),
                                   lambda: sp.build_bvh(dec, dbvh),
                                   lambda: sp.build_bvh_from_samples(pos, col, sph.count, synth.BOX_LO,
                                                                     synth.BOX_SIZE, ru, half=True, out=fused,
                                                                     bvh=fbvh)]) for _ in range(reps)])
    # algorithmic bytes per call: encode reads 16 B of centre and radius and
    # 8 B of half colour and writes the 12-byte sample; decode the reverse.
    # An eager call of a few microseconds waits on the host, so the device
    # time per call comes from replays of a captured graph of 20 calls.
    nbytes = 36 * n

    def device_ms(fn, per=20):
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(per):
                fn()
        g.replay()
        torch.cuda.synchronize()
        return float(np.median([_events(torch, [g.replay])[0] / per for _ in range(max(reps // 4, 3))]))

    enc_ms = device_ms(lambda: sp.encode_samples(sph, synth.BOX_LO, synth.BOX_SIZE, ru))
    dec_ms = device_ms(lambda: sp.decode_samples(pos, col, sph.count, synth.BOX_LO, synth.BOX_SIZE, ru, half=True,
                                                 out=dec))
    return {"spheres": n, "bytes_per_sample": 12, "bytes_per_sample_unpacked": 24,
            "algorithmic_bytes_per_call": nbytes,
            "encode_device_ms": round(enc_ms, 4), "decode_device_ms": round(dec_ms, 4),
            "encode_gb_s": round(nbytes / enc_ms / 1e6, 1), "decode_gb_s": round(nbytes / dec_ms / 1e6, 1),
            "encode_frac_of_hbm_peak": round(nbytes / enc_ms / 1e6 / 8000.0, 4),
            "decode_frac_of_hbm_peak": round(nbytes / dec_ms / 1e6 / 8000.0, 4),
            "decode_then_build_ms": round(float(np.median(tb[:, 0] + tb[:, 1])), 4),
            "build_from_samples_ms": round(float(np.median(tb[:, 2])), 4),
            "encode_ms": round(float(np.median(t[:, 0])), 4), "decode_ms": round(float(np.median(t[:, 1])), 4),
            "image_mean_abs_change": round(float(diff.mean()), 6), "image_max_abs_change": round(float(diff.max()), 4)}


def accumulate(sp, torch, synth, dev, src, sph, reps, grid=256, max_age=8):
    """Temporal accumulation at the client frame's source size: the frame seen
    from a source view 10 degrees on merged with the current frame as history.
    Algorithmic bytes: the frame read (28 B: centre + radius, half colour,
    source index) and written with its age (29 B); per history sample the
    centre and age read once (17 B); per survivor the colour and index read
    (12 B) and 29 B written; the cell map cleared (grid^3 B)."""
    vol = synth.volume_of(synth.CLIENT_FRAME)
    src1 = synth.rotated_camera(src, 10.0, 0.0)
    rgba1, depth1 = synth.raycast(vol, src1)
    frame = sp.unproject(src1, torch.from_numpy(rgba1).to(dev), torch.from_numpy(depth1).to(dev), 1.0, True)
    age = torch.zeros((sph.capacity,), dtype=torch.uint8, device=dev)
    out, out_age = sp.accumulate(frame, sph, age, synth.BOX_LO, synth.BOX_SIZE, grid, max_age)

    def call():
        sp.accumulate(frame, sph, age, synth.BOX_LO, synth.BOX_SIZE, grid, max_age, out=out, out_age=out_age)

    # one eager call is bound by the host (five launches through Python); the
    # device time comes from replays of a captured graph of the same call
    t = np.array([_events(torch, [call])[0] for _ in range(reps)])
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    graph.replay()
    torch.cuda.synchronize()
    per = 20
    dev_ms = float(np.median([_events(torch, [lambda: [graph.replay() for _ in range(per)]])[0] / per
                              for _ in range(max(reps // 4, 3))]))
    nf, nh, nm = frame.n(), sph.n(), out.n()
    kept = nm - nf
    alg = nf * (28 + 29) + nh * 17 + kept * (12 + 29) + grid ** 3
    return {"frame_samples": nf, "history_samples": nh, "merged": nm, "grid": grid, "max_age": max_age,
            "call_ms": round(float(np.median(t)), 4), "device_ms": round(dev_ms, 4), "algorithmic_bytes": int(alg),
            "gb_s": round(alg / (dev_ms * 1e-3) / 1e9, 1), "frac_of_hbm_peak": round(alg / (dev_ms * 1e-3) / 8e12, 4)}


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(rgba_np, depth_np, src, dst, scale):
    """The FP64 brute-force oracle on a bounded pixel sample of the same frame, on the host cores.
    Its spheres come from its own unprojection of the source image at the timed radius scale.  Returns
    the baseline record and what the oracle rendered (for the parity check of the timed frame)."""
    import oracle
    cr, col, idx = oracle.unproject(src, rgba_np, depth_np, scale, True)
    n = cr.shape[0]
    rng = np.random.default_rng(0)
    table = oracle.sphere_table(cr, col)
    oracle.render_table(table, dst, pixels=rng.integers(0, dst.width * dst.height, 64))  # warm
    # batches of distinct random pixels until at least 10 s of oracle time
    perm = rng.permutation(dst.width * dst.height)
    count, dt, batch, parts = 0, 0.0, 2048, []
    while dt < 10.0 and count < 400000:
        pix = perm[count:count + batch]
        t0 = time.perf_counter()
        parts.append((pix, oracle.render_table(table, dst, pixels=pix)))
        step = time.perf_counter() - t0
        dt += step
        count += pix.size
        batch = int(min(max(batch, batch * (10.0 - dt) / max(step, 1e-3)), 100000)) if dt < 10.0 else batch
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rec = {"value": round(count / dt / 1e6, 6), "unit": "Mrays/s", "cores": cores, "kind": "oracle",
           "nproc": os.cpu_count(), "cpu_model": _cpu_model(),
           "sample": f"{count} distinct random pixels of the same {dst.width}x{dst.height} frame (radius scale "
                     f"{scale}), all {n} spheres tested per ray (brute force, FP64), {dt:.1f} s"}
    render = {k: np.concatenate([r[k] for _, r in parts]) for k in ("rgba", "n", "flags", "alt_rgba", "alt_n")}
    return rec, {"pixels": np.concatenate([p for p, _ in parts]), "render": render, "spheres": (cr, col, idx)}


if __name__ == "__main__":
    main()
