"""splat_trace_noalloc (the trace whose tile-order scratch is a static device
array) against splat_trace with a caller workspace: identical images and hit
counts, bit for bit, on two calls in a row, the second on a smaller sphere
set and a smaller image.  Both images have more than 8192 tiles, so the
heaviest-first tile order, which is what uses the scratch, runs in both."""
import ctypes

import pytest
import torch

import synth
from paper_2006_14726_amd import _lib

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


def _frame(sp, work, dst):
    rgba, depth, src, _ = synth.source_image(work)
    sph = sp.unproject(src, torch.from_numpy(rgba).to(DEV), torch.from_numpy(depth).to(DEV), 1.0, True)
    bvh = sp.build_bvh(sph)
    return sph, bvh, dst


def _noalloc(sp, bvh, sph, cam, opts, out, hits):
    """The entry point through the C ABI itself."""
    lib = _lib.load()
    c, o, s, b = _lib.camera_struct(cam), opts.struct(), sph.struct(), bvh.struct()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.splat_trace_noalloc(ctypes.byref(b), ctypes.byref(s), ctypes.byref(c), ctypes.byref(o),
                                       ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(hits.data_ptr()), stream))


def test_noalloc_trace_matches_trace_twice(sp):
    big = synth.CLIENT_FRAME
    _, _, src_big, dst_big = synth.source_image(big)
    small_src = synth.source_camera(512, 512)
    dst_small = synth.rotated_camera(small_src, 12.0, 3.0, 1280, 720)
    cases = [("client frame 1920x1080", big, dst_big), ("512^2 source -> 1280x720", synth.DIFF, dst_small)]
    assert (1280 // 8) * (720 // 8) > 8192 and (1920 // 8) * (1080 // 8) > 8192
    opts = sp.TraceOptions(schedule=2)
    sizes = []
    for name, work, dst in cases:
        print(f"case {name}", flush=True)
        sph, bvh, cam = _frame(sp, work, dst)
        sizes.append(sph.n())
        ref_img, ref_hits = sp.trace(bvh, sph, cam, opts)
        H, W = cam.height, cam.width
        out = torch.full((H, W, 4), float("nan"), dtype=torch.float32, device=DEV)
        hits = torch.full((H, W), -1, dtype=torch.int32, device=DEV)
        _noalloc(sp, bvh, sph, cam, opts, out, hits)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_img), f"{name}: image differs from splat_trace"
        assert torch.equal(hits, ref_hits), f"{name}: hit counts differ from splat_trace"
        assert int((ref_hits > 0).sum()) > 1000
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_an_image_beyond_its_scratch(sp):
    sph, bvh, _ = _frame(sp, synth.TINY, None)
    lib = _lib.load()
    big = synth.source_camera(8192, 8192)
    need = lib.splat_workspace_bytes(_lib.SPLAT_OP_TRACE, 0, 8192, 8192)
    assert need > lib.splat_trace_noalloc_max_bytes()
    out = torch.empty((1, 4), dtype=torch.float32, device=DEV)  # never written: the call fails on the host
    c, o, s, b = _lib.camera_struct(big), sp.TraceOptions(schedule=2).struct(), sph.struct(), bvh.struct()
    rc = lib.splat_trace_noalloc(ctypes.byref(b), ctypes.byref(s), ctypes.byref(c), ctypes.byref(o),
                                 ctypes.c_void_p(out.data_ptr()), None, None)
    assert rc == _lib.SPLAT_ENOSPC
    assert b"scratch" in lib.splat_last_error()
