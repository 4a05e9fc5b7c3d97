"""GPU parity of temporal accumulation (splat_accumulate; Sec. 7 names keeping
samples across frames, the merge policy is this library's reading) against the
oracle's merge: the merged set must be bit for bit the oracle's (integer keep
decisions, copied bits, ages, count).  Inputs come from synth and the oracle's
own unprojection, uploaded; unused capacity is filled with NaN so that a read
past the device count shows."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import assert_parity, compare

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


def upload(sp, cr, col, src=None, cap=None, age=None):
    """Sphere set of capacity `cap` holding the given rows; the rest is NaN / 0xff junk."""
    n = cr.shape[0]
    cap = cap or max(n, 1)
    t_cr = torch.full((cap, 4), float("nan"), dtype=torch.float32)
    t_cr[:n] = torch.from_numpy(np.ascontiguousarray(cr, dtype=np.float32))
    t_col = torch.full((cap, 4), float("nan"), dtype=torch.float16 if col.dtype == np.float16 else torch.float32)
    t_col[:n] = torch.from_numpy(np.ascontiguousarray(col))
    s = sp.Spheres(t_cr.to(DEV), t_col.to(DEV), torch.tensor([n], dtype=torch.int32, device=DEV))
    if src is not None:
        t_src = torch.full((cap,), -1, dtype=torch.int32)
        t_src[:n] = torch.from_numpy(np.ascontiguousarray(src).astype(np.int64).astype(np.int32))
        s.src_index = t_src.to(DEV)
    t_age = None
    if age is not None:
        a = torch.full((cap,), 255, dtype=torch.uint8)
        a[:n] = torch.from_numpy(np.ascontiguousarray(age, dtype=np.uint8))
        t_age = a.to(DEV)
    return s, t_age


def download(s, age):
    torch.cuda.synchronize()
    n = s.n()
    out = {"cr": s.centre_radius[:n].cpu().numpy(), "rgba": s.rgba[:n].cpu().numpy(),
           "age": age[:n].cpu().numpy()}
    if s.src_index is not None:
        out["src"] = s.src_index[:n].cpu().numpy().view(np.uint32)
    return out


def assert_same(got, want, context=""):
    assert got["cr"].shape[0] == want["cr"].shape[0], f"{context}: count {got['cr'].shape[0]} vs {want['cr'].shape[0]}"
    assert np.array_equal(got["cr"].view(np.uint32), want["cr"].view(np.uint32)), f"{context}: centres differ"
    bits = np.uint16 if got["rgba"].dtype == np.float16 else np.uint32
    assert np.array_equal(got["rgba"].view(bits), np.asarray(want["rgba"]).view(bits)), f"{context}: colours differ"
    assert np.array_equal(got["age"], want["age"]), f"{context}: ages differ"
    if "src" in want and "src" in got:
        assert np.array_equal(got["src"], want["src"]), f"{context}: src differ"


def scene(seed, n_frame, n_hist, half):
    """A frame and a history that shares many cells with it (jittered copies of
    frame centres), some centres outside the box, random ages."""
    rng = np.random.default_rng(seed)
    lo, size = synth.BOX_LO, synth.BOX_SIZE

    def cols(n):
        c = rng.uniform(0, 1, (n, 4)).astype(np.float32)
        return c.astype(np.float16) if half else c

    fcr = np.zeros((n_frame, 4), dtype=np.float32)
    fcr[:, :3] = rng.uniform(lo - 0.1, lo + size + 0.1, (n_frame, 3))
    fcr[:, 3] = rng.uniform(0.002, 0.02, n_frame)
    hcr = np.zeros((n_hist, 4), dtype=np.float32)
    k = n_hist // 2
    if n_frame:
        hcr[:k, :3] = fcr[rng.integers(0, n_frame, k), :3] + rng.normal(0, 0.01, (k, 3))
    else:
        hcr[:k, :3] = rng.uniform(lo, lo + size, (k, 3))
    hcr[k:, :3] = rng.uniform(lo - 0.1, lo + size + 0.1, (n_hist - k, 3))
    hcr[:, 3] = rng.uniform(0.002, 0.02, n_hist)
    frame = {"cr": fcr, "rgba": cols(n_frame), "src": rng.integers(0, 1 << 20, n_frame).astype(np.uint32)}
    hist = {"cr": hcr, "rgba": cols(n_hist), "src": rng.integers(0, 1 << 20, n_hist).astype(np.uint32),
            "age": rng.integers(0, 7, n_hist).astype(np.uint8)}
    return frame, hist


def run(sp, frame, hist, grid, max_age, out_cap=None, f_cap=None, h_cap=None, with_src=True):
    fs, _ = upload(sp, frame["cr"], frame["rgba"], frame["src"] if with_src else None, f_cap)
    if hist is not None:
        hs, hage = upload(sp, hist["cr"], hist["rgba"], hist["src"] if with_src else None, h_cap, hist["age"])
    else:
        hs, hage = None, None
    out = None
    if out_cap is not None:
        out = sp.alloc_spheres(out_cap, DEV, frame["rgba"].dtype == np.float16)
        if not with_src:
            out.src_index = None
    m, age = sp.accumulate(fs, hs, hage, synth.BOX_LO, synth.BOX_SIZE, grid, max_age, out=out)
    return download(m, age)


@pytest.mark.parametrize("half", [True, False])
@pytest.mark.parametrize("grid", [1, 7, 32, 256])
def test_bit_exact_random(sp, half, grid):
    frame, hist = scene(3, 3000, 5000, half)
    print(f"accumulate random half={half} grid={grid}", flush=True)
    got = run(sp, frame, hist, grid, 4, f_cap=4096, h_cap=6100)
    want = oracle.accumulate(frame, hist, synth.BOX_LO, synth.BOX_SIZE, grid, 4)
    assert_same(got, want, f"grid {grid}")
    if grid == 1:
        assert got["cr"].shape[0] == 3000  # one cell: every history sample is replaced
    if grid == 256:
        assert 3000 + 1000 < got["cr"].shape[0] < 8000


def test_without_history_and_src(sp):
    frame, _ = scene(4, 2500, 0, True)
    got = run(sp, frame, None, 64, 3, f_cap=3000, with_src=False)
    assert_same(got, {"cr": frame["cr"], "rgba": frame["rgba"], "age": np.zeros(2500, np.uint8)})


def test_capacity_cut_keeps_the_newest(sp):
    frame, hist = scene(5, 2000, 6000, True)
    want = oracle.accumulate(frame, hist, synth.BOX_LO, synth.BOX_SIZE, 128, 5, capacity=4500)
    got = run(sp, frame, hist, 128, 5, out_cap=4500)
    assert want["cr"].shape[0] == 4500
    assert_same(got, want, "cut")
    tiny = run(sp, frame, hist, 128, 5, out_cap=1500)  # smaller than the frame itself
    assert_same(tiny, {k: v[:1500] for k, v in oracle.accumulate(frame, hist, synth.BOX_LO, synth.BOX_SIZE, 128,
                                                                 5).items()}, "frame cut")


def test_empty_frame_keeps_history_by_age(sp):
    frame, hist = scene(6, 0, 4000, False)
    got = run(sp, frame, hist, 64, 3, f_cap=16)
    want = oracle.accumulate(frame, hist, synth.BOX_LO, synth.BOX_SIZE, 64, 3)
    assert_same(got, want, "empty frame")
    assert got["cr"].shape[0] == int(np.sum(hist["age"] + 1 <= 3))


def test_orbit_of_frames_and_the_trace_of_the_union(sp):
    """Four source views 8 degrees apart, accumulated one after another on the
    GPU (ping-pong buffers) and by the oracle; every merged set is identical,
    and the trace of the last one matches the oracle's render of it."""
    vol = synth.volume_of(synth.CLIENT_FRAME)
    base = synth.source_camera(256, 256)
    grid, max_age = 128, 2
    g_hist = g_age = None
    o_hist = None
    for f in range(4):
        src = synth.rotated_camera(base, 8.0 * f, 2.0 * f)
        rgba, depth = synth.raycast(vol, src)
        cr, col, idx = oracle.unproject(src, rgba, depth, 1.0, True)
        frame = {"cr": cr, "rgba": col, "src": idx}
        print(f"accumulate orbit frame {f}: {cr.shape[0]} samples", flush=True)
        fs, _ = upload(sp, cr, col, idx)
        g_hist, g_age = sp.accumulate(fs, g_hist, g_age, synth.BOX_LO, synth.BOX_SIZE, grid, max_age)
        if o_hist is None:
            o_hist = oracle.accumulate(frame, {"cr": cr[:0], "rgba": col[:0], "src": idx[:0],
                                               "age": np.zeros(0, np.uint8)}, synth.BOX_LO, synth.BOX_SIZE, grid,
                                       max_age)
        else:
            o_hist = oracle.accumulate(frame, o_hist, synth.BOX_LO, synth.BOX_SIZE, grid, max_age)
        assert_same(download(g_hist, g_age), o_hist, f"frame {f}")
    n = o_hist["cr"].shape[0]
    assert n > cr.shape[0] and o_hist["age"].max() == max_age
    dst = synth.rotated_camera(base, 30.0, 4.0, 320, 240)
    bvh = sp.build_bvh(g_hist)
    img, hits = sp.trace(bvh, g_hist, dst)
    torch.cuda.synchronize()
    orc = oracle.render(o_hist["cr"], o_hist["rgba"], dst)  # every pixel
    st = compare(img.cpu().numpy().reshape(-1, 4), hits.cpu().numpy().reshape(-1), orc)
    print(f"  union: {st['pixels']} pixels, max err {st['max_err']:.2e}, exempt {st['exempt']}", flush=True)
    assert_parity(st, exempt_frac=1e-4, context="union")
    assert st["hits_checked"] > 40000


def test_full_size_client_frames(sp):
    """Two 1024 x 1024 source frames 10 degrees apart (the client frame's
    source size), merged at grid 256: the whole merged set is the oracle's."""
    vol = synth.volume_of(synth.CLIENT_FRAME)
    src0 = synth.source_camera(1024, 1024)
    frames = []
    for f in range(2):
        src = synth.rotated_camera(src0, 10.0 * f, 0.0)
        rgba, depth = synth.raycast(vol, src)
        cr, col, idx = oracle.unproject(src, rgba, depth, 1.0, True)
        frames.append({"cr": cr, "rgba": col, "src": idx})
    hist = dict(frames[0], age=np.zeros(frames[0]["cr"].shape[0], np.uint8))
    print(f"accumulate full size: {frames[1]['cr'].shape[0]} + {hist['cr'].shape[0]}", flush=True)
    got = run(sp, frames[1], hist, 256, 8, f_cap=1 << 20, h_cap=1 << 20)
    want = oracle.accumulate(frames[1], hist, synth.BOX_LO, synth.BOX_SIZE, 256, 8)
    assert_same(got, want, "full size")
    assert want["kept"].size > 1000


def test_rejects_bad_arguments(sp):
    frame, hist = scene(8, 100, 100, True)
    fs, _ = upload(sp, frame["cr"], frame["rgba"], frame["src"])
    hs, hage = upload(sp, hist["cr"], hist["rgba"], hist["src"], age=hist["age"])
    with pytest.raises(sp.SplatError):
        sp.accumulate(fs, hs, hage, synth.BOX_LO, synth.BOX_SIZE, 0, 3)
    with pytest.raises(sp.SplatError):
        sp.accumulate(fs, hs, hage, synth.BOX_LO, synth.BOX_SIZE, 64, 300)
    with pytest.raises(sp.SplatError):  # the output is the history
        sp.accumulate(fs, hs, hage, synth.BOX_LO, synth.BOX_SIZE, 64, 3, out=hs, out_age=hage)
