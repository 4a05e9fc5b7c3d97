"""GPU parity of the spheroid samples (Sec. 7 suggests smearing a sample whose
depth is uncertain over an interval along its ray; the shape, a prolate
spheroid on the source ray, is this library's reading): the unprojected set
against the oracle's, and traces through the spheroid hierarchy against the
oracle's brute-force render of the same stored samples, for every walk."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import assert_parity, compare, silhouette_pixels, tile_sample
from test_gpu_policy import marched, up

pytestmark = pytest.mark.gpu
NEVER = 2.0


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


def _ulp(a, b):
    return np.abs(a.view(np.int32).astype(np.int64) - b.view(np.int32).astype(np.int64))


@pytest.mark.parametrize("kappa", [1.0, 0.25])
def test_spheroid_unproject_matches_oracle(sp, kappa):
    rgba, depth, itv, src = marched(256)
    print(f"spheroid unproject kappa={kappa}", flush=True)
    s = sp.unproject_policy(src, up(rgba), up(depth), sp.SPLAT_RADIUS_SPHEROID, interval=up(itv),
                            interval_scale=kappa)
    torch.cuda.synchronize()
    cr, col, idx, ax = oracle.unproject_spheroids(src, rgba, depth, itv, interval_scale=kappa)
    n = s.n()
    assert n == cr.shape[0] > 5000
    g_cr = s.centre_radius[:n].cpu().numpy()
    g_ax = s.axis[:n].cpu().numpy()
    assert np.array_equal(g_cr[:, :3].view(np.uint32), cr[:, :3].view(np.uint32)), "centres differ"
    assert _ulp(g_cr[:, 3], cr[:, 3]).max() == 0, "radii differ"
    assert _ulp(g_ax, ax).max() <= 1, "axes or half-lengths differ by more than 1 ulp"
    assert np.array_equal(s.rgba[:n].cpu().numpy().view(np.uint16), col.view(np.uint16))
    assert np.array_equal(s.src_index[:n].cpu().numpy().view(np.uint32), idx)
    assert (ax[:, 3] > cr[:, 3]).mean() > 0.5  # most samples are stretched


def _random_spheroids(n, seed):
    cr, col = synth.random_spheres(n, seed=seed, r_lo=0.01, r_hi=0.04)
    rng = np.random.default_rng(seed + 100)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    h = cr[:, 3].astype(np.float64) * rng.uniform(1.0, 6.0, n)
    ax = np.concatenate([u, h[:, None]], axis=1).astype(np.float32)
    return cr, col, ax


def _trace(sp, cr, col, ax, cam, **opts):
    sph = sp.spheres_from_tensors(up(cr), up(col), up(ax))
    bvh = sp.build_bvh(sph)
    img, hits = sp.trace(bvh, sph, cam, sp.TraceOptions(**opts))
    torch.cuda.synchronize()
    return img.cpu().numpy().reshape(-1, 4), hits.cpu().numpy().reshape(-1)


@pytest.mark.parametrize("walk", [0, 1, 2])
@pytest.mark.parametrize("seed,stop", [(0, 0.99), (1, NEVER), (2, 0.0)])
def test_random_spheroid_scenes(sp, seed, stop, walk):
    cr, col, ax = _random_spheroids(400, seed)
    cam = synth.rotated_camera(synth.source_camera(57, 41), 6.0 * seed + 3.0, 2.0)
    print(f"spheroids seed={seed} stop={stop} walk={walk}", flush=True)
    g, n = _trace(sp, cr, col, ax, cam, alpha_stop=stop, walk=walk)
    st = compare(g, n, oracle.render(cr, col, cam, alpha_stop=stop, axis=ax))
    assert_parity(st, exempt_frac=None, context=f"spheroids seed {seed}")
    assert st["exempt"] <= 3
    assert st["hits_checked"] > (100 if stop == 0.0 else 300)


def test_equal_half_length_traces_the_spheres(sp):
    """With h = r the spheroid set is the sphere set: same composited hits, colours within the bar."""
    cr, col, _ = _random_spheroids(300, 7)
    ax = np.concatenate([np.tile([0.0, 0.0, 1.0], (cr.shape[0], 1)), cr[:, 3:4].astype(np.float64)],
                        axis=1).astype(np.float32)
    cam = synth.rotated_camera(synth.source_camera(48, 36), 9.0, -3.0)
    g1, n1 = _trace(sp, cr, col, ax, cam)
    sph = sp.spheres_from_tensors(up(cr), up(col))
    img, hits = sp.trace(sp.build_bvh(sph), sph, cam)
    g0, n0 = img.cpu().numpy().reshape(-1, 4), hits.cpu().numpy().reshape(-1)
    orc = oracle.render(cr, col, cam)
    ok = orc["flags"] == 0
    assert np.array_equal(n1[ok], n0[ok]) and np.abs(g1[ok] - g0[ok]).max() <= 1e-6


def test_spheroid_client_frame_sampled(sp):
    """The 1024 x 1024 source frame of the client volume, every sample smeared over its depth interval, traced
    into 1920 x 1080: one pixel per 8x8 tile and 16 silhouette tiles against the oracle, for the frustum and
    per-lane walks (which must also agree bit for bit)."""
    rgba, depth, itv, src = marched(1024)
    dst = synth.rotated_camera(src, 10.0, 3.0, 1920, 1080)
    s = sp.unproject_policy(src, up(rgba), up(depth), sp.SPLAT_RADIUS_SPHEROID, interval=up(itv),
                            interval_scale=1.0)
    bvh = sp.build_bvh(s)
    n = s.n()
    cr = s.centre_radius[:n].cpu().numpy()
    col = s.rgba[:n].cpu().numpy()
    ax = s.axis[:n].cpu().numpy()
    out = {}
    for walk in (2, 0):
        print(f"spheroid client frame walk={walk}", flush=True)
        img, hits = sp.trace(bvh, s, dst, sp.TraceOptions(walk=walk))
        torch.cuda.synchronize()
        out[walk] = (img.cpu().numpy().reshape(-1, 4), hits.cpu().numpy().reshape(-1))
    assert np.array_equal(out[0][0].view(np.uint32), out[2][0].view(np.uint32))
    assert np.array_equal(out[0][1], out[2][1])
    rng = np.random.default_rng(23)
    pix = np.unique(np.concatenate([tile_sample(dst.width, dst.height, 8, rng),
                                    silhouette_pixels(cr, dst, rng, count=8)]))
    st = compare(out[2][0][pix], out[2][1][pix], oracle.render(cr, col, dst, pixels=pix, axis=ax))
    print(f"  {st['pixels']} pixels: max err {st['max_err']:.2e}, exempt {st['exempt']}, knife {st['knife']}",
          flush=True)
    assert_parity(st, exempt_frac=1e-4, context="spheroid client frame")
    assert st["hits_checked"] > 10000


def test_spheroid_sets_refuse_soft_alpha_and_backward(sp):
    cr, col, ax = _random_spheroids(50, 3)
    cam = synth.source_camera(16, 16)
    sph = sp.spheres_from_tensors(up(cr), up(col), up(ax))
    bvh = sp.build_bvh(sph)
    with pytest.raises(sp.SplatError):
        sp.trace(bvh, sph, cam, sp.TraceOptions(mode=sp.SPLAT_ALPHA_SOFT))
