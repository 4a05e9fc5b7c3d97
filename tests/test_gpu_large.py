"""Large frame at full size: 512^3 volume with 256 blobs, 3840x2160 source,
3840x2160 targets on a 1 degree per frame orbit starting at 15 degrees, the
hierarchy rebuilt for every frame.  One pixel per 32x32 tile of frames 0, 14
and 29, plus the pixels of 16 silhouette tiles, against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import assert_parity, compare, silhouette_pixels, tile_sample

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


@pytest.fixture(scope="module")
def large():
    rgba, depth, src, _ = synth.source_image(synth.LARGE)
    cr, col, idx = oracle.unproject(src, rgba, depth, 1.0, True)
    return rgba, depth, src, cr, col, idx


def up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def test_large_unprojection(sp, large):
    rgba, depth, src, cr, col, idx = large
    print(f"large frame: {len(idx)} spheres", flush=True)
    s = sp.unproject(src, up(rgba), up(depth), 1.0, True)
    n = s.n()
    assert n == len(idx) > 3_000_000
    assert np.array_equal(s.src_index[:n].cpu().numpy().astype(np.uint32), idx)
    g = s.centre_radius[:n].cpu().numpy()
    assert np.abs(g.view(np.int32).astype(np.int64) - cr.view(np.int32)).max() <= 1
    assert np.array_equal(s.rgba[:n].cpu().numpy().view(np.uint16), col.view(np.uint16))


@pytest.mark.parametrize("frame,walk", [(0, 0), (14, 0), (29, 0), (0, 1), (0, 2), (29, 2)])
def test_large_orbit_sampled(sp, large, frame, walk):
    rgba, depth, src, cr, col, _ = large
    dst = synth.rotated_camera(src, 15.0 + frame, 0.0)
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    img, hits = sp.trace(bvh, sph, dst, sp.TraceOptions(walk=walk))
    torch.cuda.synchronize()
    rng = np.random.default_rng(frame)
    sil = silhouette_pixels(cr, dst, rng, count=8)
    pix = np.unique(np.concatenate([tile_sample(dst.width, dst.height, 32, rng), sil]))
    g = img.cpu().numpy().reshape(-1, 4)[pix]
    n = hits.cpu().numpy().reshape(-1)[pix]
    st = compare(g, n, oracle.render(cr, col, dst, pixels=pix))
    print(f"  large frame {frame}: {st['pixels']} pixels ({sil.size} in silhouette tiles), max err "
          f"{st['max_err']:.2e}, exempt {st['exempt']}, knife {st['knife']}", flush=True)
    assert_parity(st, exempt_frac=1e-4, context=f"large frame {frame}")
    assert st["pixels"] > 8100 and (n > 0).mean() > 0.2
