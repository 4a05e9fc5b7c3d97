"""GPU parity of the radius policies (splat_unproject_policy; Sec. 7 suggests
a radius varied with opacity, or a sample smeared over a depth interval along
the ray) and of the marcher's depth interval (splat_raymarch), against the
oracle.  Every input (image, depth, interval) is made on the CPU by synth or
the oracle and uploaded; the unprojected sets must match the oracle's bit for
bit, and the traced images the oracle's render of the oracle's spheres."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import assert_parity, compare, silhouette_pixels, tile_sample

pytestmark = pytest.mark.gpu
LO, SIZE = synth.BOX_LO, synth.BOX_SIZE


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


def up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


_cache = {}


def marched(size):
    """(rgba, depth, interval, src) of the client volume from a size x size source view, by the oracle."""
    if size not in _cache:
        vol = synth.volume_of(synth.CLIENT_FRAME)
        src = synth.source_camera(size, size)
        m = oracle.raymarch(vol, LO, SIZE, src)
        rgba = m["rgba"].astype(np.float32).reshape(size, size, 4)
        depth = m["depth"].astype(np.float32).reshape(size, size)
        itv = m["interval"].astype(np.float32).reshape(size, size, 2)
        _cache[size] = (rgba, depth, itv, src)
    return _cache[size]


@pytest.mark.parametrize("size", [64, 256])
def test_march_interval_matches_oracle(sp, size):
    vol = synth.volume_of(synth.CLIENT_FRAME if size == 256 else synth.TINY)
    src = synth.source_camera(size, size)
    print(f"march interval {size}", flush=True)
    rgba, depth, itv = sp.raymarch(up(vol), LO, SIZE, src, with_interval=True)
    torch.cuda.synchronize()
    g = itv.cpu().numpy().reshape(-1, 2).astype(np.float64)
    ref = oracle.raymarch(vol, LO, SIZE, src)["interval"]
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(g), fin), "interval decisions differ"
    assert fin[:, 0].sum() > 0.1 * size * size
    rel = np.abs(g[fin] - ref[fin]) / np.abs(ref[fin])
    assert rel.max() <= 1e-6, rel.max()
    # the interval holds the depth, and the other outputs are the plain marcher's
    rgba2, depth2 = sp.raymarch(up(vol), LO, SIZE, src)
    assert torch.equal(rgba, rgba2) and torch.equal(depth, depth2)
    d = depth.cpu().numpy().reshape(-1).astype(np.float64)
    ok = np.isfinite(d)
    assert np.all(g[ok, 0] <= d[ok]) and np.all(d[ok] <= g[ok, 1])


def _sets_equal(s, ref, half):
    n = s.n()
    cr, col, idx = ref
    assert n == cr.shape[0]
    g_cr = s.centre_radius[:n].cpu().numpy()
    assert np.array_equal(g_cr[:, :3].view(np.uint32), cr[:, :3].view(np.uint32)), "centres differ"
    ulp = np.abs(g_cr[:, 3].view(np.int32).astype(np.int64) - cr[:, 3].view(np.int32))
    assert ulp.max() == 0, f"radii differ by up to {ulp.max()} ulp ({(ulp > 0).sum()} spheres)"
    bits = np.uint16 if half else np.uint32
    assert np.array_equal(s.rgba[:n].cpu().numpy().view(bits), col.view(bits)), "colours differ"
    assert np.array_equal(s.src_index[:n].cpu().numpy().view(np.uint32), idx), "source indices differ"


@pytest.mark.parametrize("half", [True, False])
@pytest.mark.parametrize("mode,kw", [(0, {"radius_scale": 1.5}), (1, {"opacity_floor": 0.05}),
                                     (1, {"radius_scale": 2.0, "opacity_floor": 0.3}),
                                     (2, {"interval_scale": 1.0}), (2, {"interval_scale": 0.1})])
def test_policy_unproject_bit_exact(sp, mode, kw, half):
    rgba, depth, itv, src = marched(256)
    print(f"policy unproject mode={mode} {kw} half={half}", flush=True)
    s = sp.unproject_policy(src, up(rgba), up(depth), mode, interval=up(itv), half=half, **kw)
    torch.cuda.synchronize()
    ref = oracle.unproject_policy(src, rgba, depth, mode, interval=itv, half=half, **kw)
    assert ref[0].shape[0] > 5000
    _sets_equal(s, ref, half)


def test_footprint_policy_is_unproject(sp):
    rgba, depth, src, _ = synth.source_image(synth.CLIENT_FRAME)
    a = sp.unproject(src, up(rgba), up(depth), 1.25, True)
    b = sp.unproject_policy(src, up(rgba), up(depth), sp.SPLAT_RADIUS_FOOTPRINT, radius_scale=1.25)
    torch.cuda.synchronize()
    n = a.n()
    assert n == b.n()
    assert torch.equal(a.centre_radius[:n], b.centre_radius[:n]) and torch.equal(a.rgba[:n], b.rgba[:n])


@pytest.mark.parametrize("mode,kw", [(1, {"opacity_floor": 0.05}), (2, {"interval_scale": 0.25})])
def test_policy_client_path_full_size(sp, mode, kw):
    """The 1024 x 1024 source frame of the client volume under a policy, traced
    into 1920 x 1080: one pixel per 8x8 tile and the pixels of 16 silhouette
    tiles against the oracle's render of the oracle's spheres; the unprojected
    set is the oracle's bit for bit."""
    rgba, depth, itv, src = marched(1024)
    dst = synth.rotated_camera(src, 10.0, 3.0, 1920, 1080)
    print(f"policy client path mode={mode}", flush=True)
    s = sp.unproject_policy(src, up(rgba), up(depth), mode, interval=up(itv), **kw)
    ref = oracle.unproject_policy(src, rgba, depth, mode, interval=itv, **kw)
    _sets_equal(s, ref, True)
    bvh = sp.build_bvh(s)
    img, hits = sp.trace(bvh, s, dst)
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    pix = np.unique(np.concatenate([tile_sample(dst.width, dst.height, 8, rng),
                                    silhouette_pixels(ref[0], dst, rng, count=8)]))
    g = img.cpu().numpy().reshape(-1, 4)[pix]
    h = hits.cpu().numpy().reshape(-1)[pix]
    st = compare(g, h, oracle.render(ref[0], ref[1], dst, pixels=pix))
    print(f"  {st['pixels']} pixels: max err {st['max_err']:.2e}, exempt {st['exempt']}, knife {st['knife']}",
          flush=True)
    assert_parity(st, exempt_frac=1e-4, context=f"policy {mode}")
    assert st["hits_checked"] > 10000


def test_policy_rejects_bad_arguments(sp):
    rgba, depth, itv, src = marched(64)
    with pytest.raises(sp.SplatError):
        sp.unproject_policy(src, up(rgba), up(depth), sp.SPLAT_RADIUS_INTERVAL)  # no interval
    with pytest.raises(sp.SplatError):
        sp.unproject_policy(src, up(rgba), up(depth), sp.SPLAT_RADIUS_OPACITY, opacity_floor=0.0)
    with pytest.raises(sp.SplatError):
        sp.unproject_policy(src, up(rgba), up(depth), 7)
