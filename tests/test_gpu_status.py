"""The BVH's device status word (SPLAT_STATUS_*): clear after every build, refit and trace of a
well-formed hierarchy, for every walk and for spheroid sets; set when a trace is handed a
sphere set smaller than the one its BVH was built over (references beyond the set, which the
kernels skip); cleared again by the next build.  Every kernel ends in that case too: its walks
are bounded and its indices clamped, and the image is still written."""
import numpy as np
import pytest
import torch

import synth
from test_gpu_policy import up

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


def _scene(sp, n, seed):
    cr, col = synth.random_spheres(n, seed=seed)
    return cr, col, sp.spheres_from_tensors(up(cr), up(col))


@pytest.mark.parametrize("walk", [0, 1, 2])
def test_status_clear_after_build_refit_and_trace(sp, walk):
    cr, col, sph = _scene(sp, 3000, 11)
    cam = synth.rotated_camera(synth.source_camera(96, 80), 7.0, 2.0)
    print(f"status walk={walk}", flush=True)
    bvh = sp.build_bvh(sph)
    assert bvh.status() == 0
    sp.trace(bvh, sph, cam, sp.TraceOptions(walk=walk))
    assert bvh.status() == 0
    sp.build_bvh(sph, bvh, refit_only=True)
    sp.trace(bvh, sph, cam, sp.TraceOptions(walk=walk, kbuf=1))
    assert bvh.status() == 0


def test_status_clear_for_spheroids_and_the_client_frame(sp):
    rgba, depth, src, dst = synth.source_image(synth.CLIENT_FRAME)
    sph = sp.unproject(src, up(rgba), up(depth), 1.0, True)
    bvh = sp.build_bvh(sph)
    print("status client frame", flush=True)
    for walk in (0, 2):
        sp.trace(bvh, sph, dst, sp.TraceOptions(walk=walk))
    assert bvh.status() == 0
    cr, col = synth.random_spheres(500, seed=5, r_lo=0.01, r_hi=0.04)
    rng = np.random.default_rng(6)
    u = rng.normal(size=(500, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    ax = np.concatenate([u, cr[:, 3:4].astype(np.float64) * rng.uniform(1.0, 5.0, (500, 1))], axis=1).astype(np.float32)
    ssp = sp.spheres_from_tensors(up(cr), up(col), up(ax))
    sbvh = sp.build_bvh(ssp)
    print("status spheroids", flush=True)
    for walk in (0, 1, 2):
        sp.trace(sbvh, ssp, synth.rotated_camera(synth.source_camera(64, 48), 5.0, 1.0), sp.TraceOptions(walk=walk))
    assert sbvh.status() == 0


@pytest.mark.parametrize("walk", [0, 1, 2])
def test_status_flags_a_set_smaller_than_the_hierarchy(sp, walk):
    cr, col, sph = _scene(sp, 2000, 12)
    cam = synth.rotated_camera(synth.source_camera(64, 64), 3.0, 1.0)
    bvh = sp.build_bvh(sph)
    assert bvh.status() == 0
    small = sp.spheres_from_tensors(up(cr[:700]), up(col[:700]))
    print(f"status mismatch walk={walk}", flush=True)
    img, hits = sp.trace(bvh, small, cam, sp.TraceOptions(walk=walk))
    torch.cuda.synchronize()
    assert bvh.status() & sp.SPLAT_STATUS_CORRUPT
    assert np.isfinite(img.cpu().numpy()).all()
    sp.build_bvh(sph, bvh)
    assert bvh.status() == 0
