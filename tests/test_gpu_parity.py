"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Every input is seeded and synthetic; the oracle never consumes anything the
GPU produced: trace parity feeds both sides the same sphere arrays (from the
input generator or from the oracle's own unprojection), and the GPU's
unprojection is compared with the oracle's separately.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import (LEAF, assert_parity, bvh_core, bvh_layout, check_bvh, compare, karras_by_split, morton30,
                     silhouette_pixels, tile_sample)

pytestmark = pytest.mark.gpu

NEVER = 2.0


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


def up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_trace(sp, cr, col, cam, **opts):
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    img, hits = sp.trace(bvh, sph, cam, sp.TraceOptions(**opts))
    torch.cuda.synchronize()
    return img.cpu().numpy().reshape(-1, 4), hits.cpu().numpy().reshape(-1), sph, bvh


def ulp_diff(a, b):
    ai = a.view(np.int32).astype(np.int64)
    bi = b.view(np.int32).astype(np.int64)
    return np.abs(ai - bi)


# ---------------------------------------------------------------- unprojection

@pytest.mark.parametrize("work,scale,half", [(synth.TINY, 1.0, False), (synth.CLIENT_FRAME, 1.0, True),
                                             (synth.DIFF, 0.5, False)])
def test_unproject_matches_oracle(sp, work, scale, half):
    rgba, depth, src, _ = synth.source_image(work)
    print(f"unproject {work.name} s={scale} half={half}", flush=True)
    ocr, ocol, oidx = oracle.unproject(src, rgba, depth, scale, half)
    s = sp.unproject(src, up(rgba), up(depth), scale, half)
    torch.cuda.synchronize()
    n = s.n()
    assert n == len(oidx)
    assert np.array_equal(s.src_index[:n].cpu().numpy().astype(np.uint32), oidx)
    gcr = s.centre_radius[:n].cpu().numpy()
    assert ulp_diff(gcr, ocr).max() <= 1, "centre/radius beyond 1 ulp"
    gcol = s.rgba[:n].cpu().numpy()
    assert np.array_equal(gcol.view(np.uint16 if half else np.uint32), ocol.view(np.uint16 if half else np.uint32))


def test_unproject_invalid_pixels_are_dropped(sp):
    rng = np.random.default_rng(4)
    cam = synth.source_camera(37, 23)
    rgba = rng.uniform(0.05, 0.4, size=(23, 37, 4)).astype(np.float32)
    rgba[..., 3] = rng.uniform(0.5, 1.0, size=(23, 37))
    depth = rng.uniform(1.5, 2.5, size=(23, 37)).astype(np.float32)
    flat = depth.ravel()
    flat[::5] = np.inf
    flat[1::7] = np.nan
    flat[2::11] = 0.0
    flat[3::13] = -2.0
    rgba.reshape(-1, 4)[4::17, 3] = 0.0
    ocr, ocol, oidx = oracle.unproject(cam, rgba, depth, 1.0, True)
    s = sp.unproject(cam, up(rgba), up(depth), 1.0, True)
    n = s.n()
    assert n == len(oidx) and np.array_equal(s.src_index[:n].cpu().numpy().astype(np.uint32), oidx)


# ---------------------------------------------------------------- BVH

@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 2047, 2048, 2049, 5000])
def test_bvh_structure(sp, n):
    cr, col = synth.random_spheres(n, seed=100 + n)
    print(f"bvh n={n}", flush=True)
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    torch.cuda.synchronize()
    info = check_bvh(bvh.mem.cpu().numpy(), bvh.capacity, cr, col[:, 3])
    assert info["n"] == n


def test_bvh_with_duplicate_codes(sp):
    cr, col = synth.adversarial_spheres(3)
    cr = np.concatenate([cr, np.repeat(cr[:1], 300, axis=0)])  # many identical Morton codes
    col = np.concatenate([col, np.repeat(col[:1], 300, axis=0)])
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    torch.cuda.synchronize()
    check_bvh(bvh.mem.cpu().numpy(), bvh.capacity, cr, col[:, 3])


def _built(sp, cr, col):
    """Build through the C ABI with a workspace of the test's own, so that the
    sorted keys (the first array of the build workspace) can be read back."""
    sph = sp.spheres_from_tensors(up(cr), up(col))
    lib = sp.load_library()
    ws = torch.zeros(lib.splat_workspace_bytes(sp._lib.SPLAT_OP_BUILD, sph.capacity, 0, 0), dtype=torch.uint8,
                     device="cuda:0")
    bvh = sp.build_bvh(sph, ws=ws)
    torch.cuda.synchronize()
    mem = bvh.mem.cpu().numpy()
    n = cr.shape[0]
    keys = ws[:4 * n].cpu().numpy().view(np.uint32)
    return mem, keys


def _clustered(n, seed, dup=0):
    cr, col = synth.random_spheres(n, seed=seed, r_lo=0.002, r_hi=0.01)
    if dup:  # equal Morton codes: the sorted position breaks the tie
        cr[-dup:, :3] = cr[0, :3] + np.float32(1e-6) * np.arange(dup, dtype=np.float32)[:, None]
    return cr, col


@pytest.mark.parametrize("n,dup", [(2, 0), (3, 0), (17, 0), (64, 0), (64, 20), (1000, 0), (5000, 300)])
def test_sort_is_stable_sort_of_morton_codes(sp, n, dup):
    """The radix sort against a stable sort on the host: the scene's centre box
    in the header is the exact min/max of the centres, the keys come out as the
    host's 30-bit codes of that box in ascending order, and equal codes keep
    the order of their sphere ids."""
    cr, col = _clustered(n, 500 + n, dup)
    mem, keys = _built(sp, cr, col)
    hdr = mem[:256].view(np.float32)
    cen_lo, cen_hi = hdr[8:11], hdr[11:14]
    assert np.array_equal(cen_lo, cr[:, :3].min(axis=0)) and np.array_equal(cen_hi, cr[:, :3].max(axis=0))
    codes = morton30(cr, cen_lo, cen_hi)
    order = np.argsort(codes, kind="stable")
    lay = bvh_layout(n)
    leaf_ids = mem[lay["leaf_ids"]: lay["leaf_ids"] + 4 * n].view(np.uint32)
    assert np.array_equal(leaf_ids, order.astype(np.uint32)), "sorted ids differ from a stable sort"
    assert np.array_equal(keys, codes[order]), "sorted keys differ"
    if dup:
        assert np.unique(codes).size < n


@pytest.mark.parametrize("n,dup", [(2, 0), (3, 0), (17, 0), (33, 10), (64, 0), (64, 40), (2000, 0), (5000, 300)])
def test_karras_tree_equals_recursive_split(sp, n, dup):
    """The hierarchy against its definition: every internal node's two child
    references and split axis equal those of a recursive split of the sorted
    (code, position) pairs at their highest differing bit."""
    cr, col = _clustered(n, 900 + n, dup)
    mem, keys = _built(sp, cr, col)
    lay = bvh_layout(n)
    leaf_ids = mem[lay["leaf_ids"]: lay["leaf_ids"] + 4 * n].view(np.uint32)
    ref = karras_by_split(keys, leaf_ids)
    assert len(ref) == n - 1
    f = mem[lay["nodes"]: lay["nodes"] + (n - 1) * 64].view(np.uint32).reshape(n - 1, 16)
    for node, (left, right, axis) in ref.items():
        got = (int(f[node, 12]), int(f[node, 13]), int(f[node, 14]))
        assert got == (left, right, axis), f"node {node}: {got} vs split {(left, right, axis)}"
    assert sum(1 for v in ref.values() for r in v[:2] if r & LEAF) == n


def test_build_is_deterministic(sp):
    """Bit-identical hierarchy over repeated builds (catches ordering races in sort and refit)."""
    rgba, depth, src, _ = synth.source_image(synth.DIFF)
    s = sp.unproject(src, up(rgba), up(depth), 1.0, False)
    bvh = sp.build_bvh(s)
    ref = bvh_core(bvh.mem, bvh.capacity)
    for _ in range(20):
        sp.build_bvh(s, bvh)
        assert torch.equal(ref, bvh_core(bvh.mem, bvh.capacity))
    n = s.n()
    cr = s.centre_radius[:n].cpu().numpy()
    col = s.rgba[:n].cpu().numpy()
    check_bvh(bvh.mem.cpu().numpy(), bvh.capacity, cr, col[:, 3])


def test_refit_matches_full_build(sp):
    cr, col = synth.random_spheres(3000, seed=7)
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    sph.centre_radius[:, 3] *= 1.5
    sph.rgba[:, 3] *= 0.5
    sp.build_bvh(sph, bvh, refit_only=True)
    fresh = sp.build_bvh(sph)
    torch.cuda.synchronize()
    assert torch.equal(bvh_core(bvh.mem, bvh.capacity), bvh_core(fresh.mem, fresh.capacity))
    # the refit rewrites the 4-wide nodes the trace reads
    w0 = bvh_layout(bvh.capacity)["wide"]
    w1 = w0 + (3000 - 1) * 128
    assert torch.equal(bvh.mem[w0:w1], fresh.mem[w0:w1])
    check_bvh(bvh.mem.cpu().numpy(), bvh.capacity, sph.centre_radius.cpu().numpy(), sph.rgba[:, 3].cpu().numpy())


# ---------------------------------------------------------------- trace

@pytest.mark.parametrize("walk", [0, 1, 2])
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("mode,stop", [(0, 0.99), (0, NEVER), (0, 0.0), (1, 0.99), (1, NEVER)])
def test_trace_random_scenes(sp, seed, mode, stop, walk):
    cr, col = synth.random_spheres(200, seed=seed, r_lo=0.02, r_hi=0.12)
    cam = synth.rotated_camera(synth.source_camera(45, 37), 8.0 * seed, 3.0)
    print(f"random seed={seed} mode={mode} stop={stop} walk={walk}", flush=True)
    g, n, _, _ = gpu_trace(sp, cr, col, cam, alpha_stop=stop, mode=mode, walk=walk)
    orc = oracle.render(cr, col, cam, alpha_stop=stop, mode=mode)
    st = compare(g, n, orc)
    assert_parity(st, exempt_frac=None, context=f"seed {seed}")
    assert st["exempt"] <= 3
    assert st["hits_checked"] > (100 if stop == 0.0 else 200)


@pytest.mark.parametrize("walk", [0, 1, 2])
@pytest.mark.parametrize("half", [False, True])
def test_trace_adversarial_scene(sp, half, walk):
    cr, col = synth.adversarial_spheres(5)
    if half:
        col = synth.to_half_rgba(col)
    cam = synth.rotated_camera(synth.source_camera(64, 48), 12.0, -4.0)
    for stop in (0.99, NEVER):
        g, n, _, _ = gpu_trace(sp, cr, col, cam, alpha_stop=stop, walk=walk)
        st = compare(g, n, oracle.render(cr, col, cam, alpha_stop=stop))
        assert_parity(st, exempt_frac=None, context=f"adversarial stop={stop}")


@pytest.mark.parametrize("yaw", [0.0, 180.0])
def test_every_direction_sign_pattern(sp, yaw):
    """A 90-degree view along -z (yaw 0) or +z (yaw 180) of odd size: its four
    quadrants give four of the eight sign patterns of the ray directions, so
    the two views give all eight to the per-lane walk's box test, and the
    tiles on the middle row and column mix signs, or (the middle column,
    x + 1/2 = W/2) hold a direction component of exactly 0.  The per-lane walk
    must match the packet walk bit for bit, and the oracle on every pixel."""
    cr, col = synth.random_spheres(1500, seed=7, r_lo=0.01, r_hi=0.05)
    # the eye 0.45 from the centre, outside every sphere (centres within 0.2 of it, radii below 0.05)
    cam = synth.rotated_camera(synth.source_camera(67, 53, fov_y_deg=90.0, distance=0.45), yaw, 0.0)
    f = np.array(cam.forward)
    assert abs(abs(f[2]) - 1.0) < 1e-12
    print(f"sign patterns yaw={yaw}", flush=True)
    out = {}
    for walk in (0, 1, 2):
        out[walk] = gpu_trace(sp, cr, col, cam, walk=walk)[:2]
    for walk in (1, 2):
        assert np.array_equal(out[0][0].view(np.uint32), out[walk][0].view(np.uint32)), walk
        assert np.array_equal(out[0][1], out[walk][1]), walk
    st = compare(out[0][0], out[0][1], oracle.render(cr, col, cam))
    assert_parity(st, exempt_frac=None, context=f"sign patterns yaw={yaw}")
    assert st["hits_checked"] > 3000


@pytest.mark.parametrize("stop", [0.99, NEVER])
def test_column_along_the_view_ray(sp, stop):
    """16384 spheres strung along the central ray of a 15x15 view: every box on
    the way is hit, so the near-first walk pushes three siblings per wide level
    and a lane's own stack (16 entries) overflows; those lanes are then settled
    by the packet walk.  Both walks must match the oracle, and each other."""
    rng = np.random.default_rng(21)
    cam = synth.source_camera(15, 15)
    n = 16384
    t = rng.uniform(1.0, 3.0, n)
    e, f = np.array(cam.eye), np.array(cam.forward)
    r_, u_ = np.array(cam.right), np.array(cam.up)
    c = e + t[:, None] * f + rng.normal(0, 0.002, (n, 1)) * r_ + rng.normal(0, 0.002, (n, 1)) * u_
    cr = np.concatenate([c, rng.uniform(0.01, 0.03, (n, 1))], axis=1).astype(np.float32)
    col = np.concatenate([rng.uniform(0, 1, (n, 3)), np.full((n, 1), 0.05)], axis=1).astype(np.float32)
    orc = oracle.render(cr, col, cam, alpha_stop=stop)
    out = {}
    for walk in (0, 1, 2):
        print(f"column stop={stop} walk={walk}", flush=True)
        g, h, _, _ = gpu_trace(sp, cr, col, cam, alpha_stop=stop, walk=walk)
        assert_parity(compare(g, h, orc), exempt_frac=None, context=f"column walk={walk}")
        out[walk] = (g, h)
    assert int(out[0][1].max()) > (1000 if stop == NEVER else 50)
    for walk in (1, 2):
        assert np.array_equal(out[0][0], out[walk][0]) and np.array_equal(out[0][1], out[walk][1]), walk


def test_heaviest_first_order_matches_other_schedules(sp):
    """Above the tile threshold the heaviest-first order is computed and used;
    the image and hit counts match schedules 0 and 1 bit for bit, for both
    walks, and the oracle on sampled pixels."""
    cr, col = synth.random_spheres(6000, seed=31, r_lo=0.004, r_hi=0.03)
    cam = synth.rotated_camera(synth.source_camera(1024, 768), 9.0, 4.0)
    assert (1024 // 8) * (768 // 8) > 8192
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    ref = None
    for walk in (0, 1, 2):
        for sched in (2, 0, 1):
            img, hits = sp.trace(bvh, sph, cam, sp.TraceOptions(schedule=sched, walk=walk))
            if ref is None:
                ref = (img.clone(), hits.clone())
            else:
                assert torch.equal(img, ref[0]) and torch.equal(hits, ref[1]), (walk, sched)
    pix = np.random.default_rng(3).integers(0, cam.width * cam.height, 3000)
    g = ref[0].cpu().numpy().reshape(-1, 4)[pix]
    n = ref[1].cpu().numpy().reshape(-1)[pix]
    st = compare(g, n, oracle.render(cr, col, cam, pixels=pix))
    assert_parity(st, exempt_frac=None, context="heaviest first")
    assert st["hits_checked"] > 300


def test_result_independent_of_kbuf_and_tile(sp):
    """The hit buffer size and the tile shape change the schedule, never the image."""
    cr, col = synth.random_spheres(400, seed=11, r_lo=0.03, r_hi=0.15)
    cam = synth.rotated_camera(synth.source_camera(67, 45), 6.0, 2.0)
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    ref = None
    for stop in (0.99, NEVER):
        ref = None
        for k in (1, 2, 4, 6, 8, 16):
            for tile in ((8, 8), (16, 4), (32, 2)):
                for walk in (0, 1, 2):
                    for sched in (0, 1, 2):
                        o = sp.TraceOptions(alpha_stop=stop, kbuf=k, tile=tile, walk=walk, schedule=sched)
                        img, hits = sp.trace(bvh, sph, cam, o)
                        if ref is None:
                            ref = (img.clone(), hits.clone())
                            if stop == NEVER:
                                assert int(hits.max()) > 16  # several restarts at k = 1, 2, 4, 6, 8
                        else:
                            assert torch.equal(img, ref[0]) and torch.equal(hits, ref[1]), (k, tile, walk, sched)


def test_tiny_config_full_frame(sp):
    """64x64 source, radius = 1 footprint, target rotated 5 deg, all float32: every pixel."""
    rgba, depth, src, dst = synth.source_image(synth.TINY)
    cr, col, _ = oracle.unproject(src, rgba, depth, 1.0, False)
    g, n, _, _ = gpu_trace(sp, cr, col, dst)
    st = compare(g, n, oracle.render(cr, col, dst))
    assert_parity(st, context="tiny")
    assert st["hits_checked"] > 100


@pytest.mark.parametrize("scale,walk", [(0.5, 0), (1.0, 0), (2.0, 0), (1.0, 1), (2.0, 1), (0.5, 2), (1.0, 2),
                                        (2.0, 2)])
def test_client_frame_sampled(sp, scale, walk):
    """1024^2 source -> 1920x1080 after 10 deg yaw + 3 deg pitch, half colours, full-size launch
    with the default schedule; the oracle checks one random pixel in every 8x8 tile (32,400) and
    every pixel of the 32 silhouette tiles (edge-on sheet, coverage edges)."""
    rgba, depth, src, dst = synth.source_image(synth.CLIENT_FRAME)
    cr, col, _ = oracle.unproject(src, rgba, depth, scale, True)
    print(f"client frame s={scale} walk={walk}: {len(cr)} spheres", flush=True)
    g, n, _, _ = gpu_trace(sp, cr, col, dst, walk=walk)
    rng = np.random.default_rng(int(scale * 10))
    sil = silhouette_pixels(cr, dst, rng)
    pix = np.unique(np.concatenate([tile_sample(dst.width, dst.height, 8, rng), sil]))
    orc = oracle.render(cr, col, dst, pixels=pix)
    st = compare(g[pix], n[pix], orc)
    print(f"  {st['pixels']} pixels ({sil.size} in silhouette tiles): max err {st['max_err']:.2e}, "
          f"exempt {st['exempt']}, knife {st['knife']}", flush=True)
    assert_parity(st, exempt_frac=1e-4, context=f"client s={scale}")
    assert st["pixels"] > 33000 and (n[pix] > 0).mean() > 0.3


def test_identity_reprojection_on_gpu(sp):
    rgba, depth, src, _ = synth.source_image(synth.TINY)
    s = sp.unproject(src, up(rgba), up(depth), 0.01, False)
    bvh = sp.build_bvh(s)
    img, hits = sp.trace(bvh, s, src)
    img = img.cpu().numpy()
    has = np.isfinite(depth) & (depth > 0)
    assert np.abs(img[has] - rgba[has]).max() <= 1e-6
    assert np.all(img[~has] == 0)
    assert np.all(hits.cpu().numpy()[has] == 1)


def test_alpha_monotone_in_t_max_on_gpu(sp):
    rgba, depth, src, dst = synth.source_image(synth.TINY)
    s = sp.unproject(src, up(rgba), up(depth), 1.0, False)
    bvh = sp.build_bvh(s)
    prev = None
    for t_max in (1.0, 1.9, 2.1, 2.3, 2.6, float("inf")):
        img, _ = sp.trace(bvh, s, dst, sp.TraceOptions(t_max=t_max))
        A = img[..., 3]
        assert bool((img[..., :3] <= A[..., None] + 1e-6).all()) and bool((A <= 1 + 1e-6).all())
        if prev is not None:
            assert bool((A >= prev).all())
        prev = A


def test_empty_and_single_sphere(sp):
    cam = synth.rotated_camera(synth.source_camera(19, 13), 3.0)
    empty = sp.alloc_spheres(16, "cuda:0", half=False)
    bvh = sp.build_bvh(empty)
    img, hits = sp.trace(bvh, empty, cam)
    assert float(img.abs().max()) == 0.0 and int(hits.max()) == 0
    cr = np.array([[0.5, 0.5, 0.5, 0.2]], dtype=np.float32)
    col = np.array([[0.2, 0.4, 0.6, 0.7]], dtype=np.float32)
    g, n, _, _ = gpu_trace(sp, cr, col, cam)
    assert_parity(compare(g, n, oracle.render(cr, col, cam)), exempt_frac=None)
    assert n.max() == 1


@pytest.mark.parametrize("w,h", [(1, 1), (7, 5), (65, 3), (3, 130)])
def test_ragged_image_sizes(sp, w, h):
    cr, col = synth.random_spheres(150, seed=w * h, r_lo=0.03, r_hi=0.15)
    cam = synth.rotated_camera(synth.source_camera(w, h), 4.0)
    for tile in ((8, 8), (32, 2)):
        g, n, _, _ = gpu_trace(sp, cr, col, cam, tile=tile)
        assert_parity(compare(g, n, oracle.render(cr, col, cam)), exempt_frac=None)


def test_errors_on_device(sp):
    cam = synth.source_camera(8, 8)
    s = sp.alloc_spheres(10, "cuda:0")
    with pytest.raises(sp.SplatError) as e:
        sp.unproject(cam, up(np.zeros((8, 8, 4), np.float32)), up(np.zeros((8, 8), np.float32)), 1.0, out=s)
    assert e.value.code == 2


def test_trace_kernel_events(sp):
    """Events passed in the options bracket the trace kernel alone: they time
    it (after the tile ordering) and change nothing in the result."""
    cr, col = synth.random_spheres(6000, seed=31, r_lo=0.004, r_hi=0.03)
    cam = synth.rotated_camera(synth.source_camera(1024, 768), 9.0, 4.0)
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    img0, hits0 = sp.trace(bvh, sph, cam)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    b.record()
    torch.cuda.synchronize()
    img1, hits1 = sp.trace(bvh, sph, cam, sp.TraceOptions(events=(a.cuda_event, b.cuda_event)))
    torch.cuda.synchronize()
    assert torch.equal(img0, img1) and torch.equal(hits0, hits1)
    assert 0.0 < a.elapsed_time(b) < 1000.0
