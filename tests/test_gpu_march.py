"""GPU parity of the server ray marcher (splat_raymarch, the stage before the
path, Sec. 4.1) against the oracle's FP64 marcher, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from test_oracle_march_pins import _axis_camera

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


def up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def march(sp, vol, lo, size, cam, **kw):
    rgba, depth = sp.raymarch(up(vol), lo, size, cam, **kw)
    torch.cuda.synchronize()
    return rgba.cpu().numpy().reshape(-1, 4).astype(np.float64), depth.cpu().numpy().reshape(-1).astype(np.float64)


def check(g_rgba, g_depth, ref, context=""):
    """RGBA to float rounding (outputs are float, the oracle is double); the
    depth decision identical and its value to float rounding."""
    err = np.abs(g_rgba - ref["rgba"]).max() if len(g_rgba) else 0.0
    assert err <= 1e-6, f"{context}: rgba off by {err}"
    fin = np.isfinite(ref["depth"])
    assert np.array_equal(np.isfinite(g_depth), fin), f"{context}: depth decisions differ"
    if fin.any():
        rel = np.abs(g_depth[fin] - ref["depth"][fin]) / np.abs(ref["depth"][fin])
        assert rel.max() <= 1e-6, f"{context}: depth off by {rel.max()}"
    return int(fin.sum())


def test_march_tiny_full_frame(sp):
    vol = synth.volume_of(synth.TINY)
    _, _, src, _ = synth.source_image(synth.TINY)
    print("march tiny", flush=True)
    g, d = march(sp, vol, synth.BOX_LO, synth.BOX_SIZE, src)
    assert check(g, d, oracle.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src), "tiny") > 400


def test_march_client_source_sampled(sp):
    """256^3 volume, 64 blobs, the 1024^2 source view: one pixel per 32x32
    tile plus 512 random pixels against the oracle."""
    vol = synth.volume_of(synth.CLIENT_FRAME)
    _, _, src, _ = synth.source_image(synth.CLIENT_FRAME)
    print("march client source", flush=True)
    g, d = march(sp, vol, synth.BOX_LO, synth.BOX_SIZE, src)
    rng = np.random.default_rng(7)
    W, H = src.width, src.height
    tx, ty = np.meshgrid(np.arange(0, W, 32), np.arange(0, H, 32))
    px = np.minimum(tx + rng.integers(0, 32, tx.shape), W - 1)
    py = np.minimum(ty + rng.integers(0, 32, ty.shape), H - 1)
    pix = np.unique(np.concatenate([(py * W + px).ravel(), rng.integers(0, W * H, 512)]))
    ref = oracle.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src, pixels=pix)
    assert check(g[pix], d[pix], ref, "client source") > 300


def test_march_feeds_unproject_like_the_input_generator(sp):
    """The GPU image matches the input generator's source image (separate code,
    same rules) to float rounding, and unprojects to the same sphere count."""
    vol = synth.volume_of(synth.TINY)
    rgba, depth, src, _ = synth.source_image(synth.TINY)
    grgba, gdepth = sp.raymarch(up(vol), synth.BOX_LO, synth.BOX_SIZE, src)
    torch.cuda.synchronize()
    assert np.abs(grgba.cpu().numpy() - rgba).max() < 1e-6
    assert np.array_equal(np.isfinite(gdepth.cpu().numpy()), np.isfinite(depth))
    a = sp.unproject(src, grgba, gdepth, 1.0, True)
    b = sp.unproject(src, up(rgba), up(depth), 1.0, True)
    torch.cuda.synchronize()
    assert a.n() == b.n() > 0


@pytest.mark.parametrize("case", ["inside", "away", "single_voxel", "ragged", "coarse_step"])
def test_march_edge_cases(sp, case):
    lo, size = -0.25, 1.5
    centre = lo + size / 2
    vol = synth.volume_of(synth.TINY)
    kw = {}
    if case == "inside":
        cam = _axis_camera(33, 17, (centre, centre, centre), (0.3, -0.2, -1.0))
    elif case == "away":
        cam = _axis_camera(9, 7, (5.0, 5.0, 5.0), (1.0, 1.0, 1.0))
    elif case == "single_voxel":
        vol = np.full((1, 1, 1), 7.5, dtype=np.float32)
        cam = _axis_camera(13, 11, (centre, centre, 3.0), (0.0, 0.0, -1.0))
    elif case == "ragged":
        _, _, src, _ = synth.source_image(synth.TINY)
        cam = synth.rotated_camera(src, 3.0, 2.0, 67, 29)
    else:
        _, _, cam, _ = synth.source_image(synth.TINY)
        kw = {"step": 2.0}
    print(f"march edge {case}", flush=True)
    g, d = march(sp, vol, lo, size, cam, **kw)
    ref = oracle.raymarch(vol, lo, size, cam, **kw)
    check(g, d, ref, case)
    if case == "away":
        assert np.all(g == 0) and np.all(np.isinf(d))


def test_march_rejects_a_tiny_step(sp):
    vol = synth.volume_of(synth.TINY)
    _, _, src, _ = synth.source_image(synth.TINY)
    with pytest.raises(sp.SplatError):
        sp.raymarch(up(vol), synth.BOX_LO, synth.BOX_SIZE, src, step=0.001)
