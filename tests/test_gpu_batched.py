"""Batched persistent trace: bit-identical to per-job plain launches, stable
under HIP-graph replay, sampled pixels against the oracle, and the
autotuner."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import assert_parity, compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


def up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.fixture(scope="module")
def small_batch():
    frames = synth.batch_frames(n_frames=7, meta_seed=9, src_sizes=(48, 64, 96),
                                dst_sizes=((80, 60), (70, 45), (130, 66)))
    out = []
    for fr in frames:
        rgba, depth, src, dsts = synth.batch_frame_images(fr, vol_n=32)
        out.append((rgba, depth, src, dsts))
    return out


def make_renderer(sp, batch, **kw):
    from paper_2006_14726_amd.batched import BatchedRenderer, Frame
    frames = [Frame(up(r), up(d), s, dsts) for r, d, s, dsts in batch]
    return BatchedRenderer(frames, **kw)


def snapshot(r):
    return [[(o.clone(), h.clone()) for o, h in views] for views in r.outputs]


def assert_same(a, b):
    for va, vb in zip(a, b):
        for (oa, ha), (ob, hb) in zip(va, vb):
            assert torch.equal(oa, ob) and torch.equal(ha, hb)


GRID = -1  # one workgroup per (job, tile)


@pytest.mark.parametrize("kbuf,tile,waves,walk", [(6, (8, 8), 0, 0), (8, (8, 8), 0, 1), (4, (16, 4), 97, 0),
                                                  (1, (32, 2), 3, 1), (6, (8, 8), 0, 2), (2, (16, 4), 97, 2),
                                                  (6, (8, 8), GRID, 2), (8, (8, 8), GRID, 0), (1, (32, 2), GRID, 1)])
def test_batched_equals_sequential(sp, small_batch, kbuf, tile, waves, walk):
    r = make_renderer(sp, small_batch, half=True, opts=sp.TraceOptions(kbuf=kbuf, tile=tile, walk=walk), waves=waves)
    assert r.n_jobs >= 7
    r.run_sequential()
    ref = snapshot(r)
    for views in r.outputs:
        for o, h in views:
            o.zero_()
            h.zero_()
    r.run()
    torch.cuda.synchronize()
    assert_same(snapshot(r), ref)
    assert sum(int(h.sum()) for views in ref for _, h in views) > 100


def test_build_lanes_match_one_stream(sp, small_batch):
    """Frames built on several streams (eager and as parallel graph branches)
    give the same hierarchies and outputs as the builds on one stream."""
    one = make_renderer(sp, small_batch, half=True, build_streams=1)
    assert len(one.lanes) == 1 and not one.streams
    one.run()
    torch.cuda.synchronize()
    ref = snapshot(one)
    four = make_renderer(sp, small_batch, half=True, build_streams=4)
    assert len(four.lanes) == 4 and sorted(i for lane in four.lanes for i in lane) == list(range(len(small_batch)))
    four.run()
    torch.cuda.synchronize()
    assert_same(snapshot(four), ref)
    for a, b in zip(one.bvhs, four.bvhs):
        assert torch.equal(a.mem[:64], b.mem[:64])  # header: root, counts, scene box
    four.capture()
    for it in range(3):
        for views in four.outputs:
            for o, h in views:
                o.fill_(float(it + 2))
                h.fill_(-1)
        for s in four.spheres:
            s.centre_radius.fill_(float("nan"))
        torch.cuda.synchronize()
        four.replay()
        torch.cuda.synchronize()
        assert_same(snapshot(four), ref)
        _ = torch.ones(1000, device="cuda:0").sum().item()


def test_graph_replay_matches_eager(sp, small_batch):
    r = make_renderer(sp, small_batch, half=True)
    r.run()
    torch.cuda.synchronize()
    ref = snapshot(r)
    r.capture()
    for it in range(3):
        for views in r.outputs:
            for o, h in views:
                o.fill_(float(it + 1))
                h.fill_(-1)
        torch.cuda.synchronize()
        r.replay()
        torch.cuda.synchronize()
        assert_same(snapshot(r), ref)
        _ = torch.ones(1000, device="cuda:0").sum().item()  # eager work between replays


def test_batched_output_against_oracle(sp, small_batch):
    r = make_renderer(sp, small_batch, half=True)
    r.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(3)
    for fi in (0, 3, 6):
        s = r.spheres[fi]
        n = s.n()
        cr = s.centre_radius[:n].cpu().numpy()
        col = s.rgba[:n].cpu().numpy()
        # the oracle traces its own unprojection of the same source image
        rgba, depth, src, dsts = small_batch[fi]
        ocr, ocol, _ = oracle.unproject(src, rgba, depth, 1.0, True)
        assert np.array_equal(ocol.view(np.uint16), col.view(np.uint16))
        assert np.abs(ocr.view(np.int32).astype(np.int64) - cr.view(np.int32)).max() <= 1
        for vi, cam in enumerate(dsts):
            img, hits = r.outputs[fi][vi]
            pix = rng.integers(0, cam.width * cam.height, 300)
            g = img.cpu().numpy().reshape(-1, 4)[pix]
            h = hits.cpu().numpy().reshape(-1)[pix]
            assert_parity(compare(g, h, oracle.render(ocr, ocol, cam, pixels=pix)), exempt_frac=None)


def test_autotuner_picks_a_valid_schedule(sp, small_batch, tmp_path, monkeypatch):
    from paper_2006_14726_amd import autotune
    monkeypatch.setenv("SPLAT_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    rgba, depth, src, dsts = small_batch[2]
    s = sp.unproject(src, up(rgba), up(depth), 1.0, True)
    bvh = sp.build_bvh(s)
    opts, rec = autotune.tune_trace(bvh, s, dsts[0])
    assert opts.kbuf in (6, 8) and opts.walk in (0, 1) and len(rec["all_ms"]) == len(autotune.TRACE_CANDIDATES)
    ref, _ = sp.trace(bvh, s, dsts[0])
    got, _ = sp.trace(bvh, s, dsts[0], opts)
    assert torch.equal(ref, got)
    again, rec2 = autotune.tune_trace(bvh, s, dsts[0])  # from the cache
    assert rec2["kbuf"] == rec["kbuf"]
    r = make_renderer(sp, small_batch, half=True)
    r.run_sequential()
    ref_out = snapshot(r)
    best = autotune.tune_batched(r)
    assert best["waves"] > 0 or best["waves"] == GRID
    r.run()
    torch.cuda.synchronize()
    assert_same(snapshot(r), ref_out)


def test_full_size_job_against_oracle(sp):
    """A batch job at the batched workload's largest size, a 2048^2 source of the client volume
    traced into 1920x1080, in the grid launch with the frustum walk: one pixel per 32x32 tile
    against the oracle's trace of its own unprojection of the same image."""
    from paper_2006_14726_amd.batched import GRID
    w = synth.Workload("client-2048sq", 256, 64, 2, 2048, 2048, 1920, 1080, 10.0, 3.0)
    rgba, depth, src, dst = synth.source_image(w)
    print("full-size batched job", flush=True)
    r = make_renderer(sp, [(rgba, depth, src, [dst])], half=True, opts=sp.TraceOptions(walk=2), waves=GRID)
    r.run()
    torch.cuda.synchronize()
    ocr, ocol, _ = oracle.unproject(src, rgba, depth, 1.0, True)
    s = r.spheres[0]
    n = s.n()
    assert n == ocr.shape[0] > 2_000_000
    assert np.array_equal(ocol.view(np.uint16), s.rgba[:n].cpu().numpy().view(np.uint16))
    assert np.abs(ocr.view(np.int32).astype(np.int64) - s.centre_radius[:n].cpu().numpy().view(np.int32)).max() <= 1
    img, hits = r.outputs[0][0]
    rng = np.random.default_rng(8)
    ty, tx = np.meshgrid(np.arange(0, dst.height, 32), np.arange(0, dst.width, 32), indexing="ij")
    px = np.minimum(tx + rng.integers(0, 32, tx.shape), dst.width - 1)
    py = np.minimum(ty + rng.integers(0, 32, ty.shape), dst.height - 1)
    pix = np.unique((py * dst.width + px).ravel())
    g = img.cpu().numpy().reshape(-1, 4)[pix]
    h = hits.cpu().numpy().reshape(-1)[pix]
    # the oracle traces its own unprojection (equal to the GPU's to 1 ulp in the radius)
    st = compare(g, h, oracle.render(ocr, ocol, dst, pixels=pix))
    print(f"  {st['pixels']} pixels: max err {st['max_err']:.2e}, exempt {st['exempt']}", flush=True)
    assert_parity(st, exempt_frac=1e-4, context="2048^2 batched job")
    assert st["hits_checked"] > 500
