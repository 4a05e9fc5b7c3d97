"""GPU parity of the sample codec (splat_encode_samples / splat_decode_samples,
the wire format of Sec. 4.1 and Sec. 5) against the oracle's codec, and the
client path run on decoded samples."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import assert_parity, bvh_core, bvh_layout, compare

pytestmark = pytest.mark.gpu
LO, SIZE = synth.BOX_LO, synth.BOX_SIZE


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


@pytest.fixture(scope="module")
def client(sp):
    """The client frame's spheres from the oracle's unprojection (CPU), uploaded:
    both sides of every comparison start from the same oracle-made arrays."""
    rgba, depth, src, dst = synth.source_image(synth.CLIENT_FRAME)
    cr, col, _ = oracle.unproject(src, rgba, depth, 1.0, True)
    s = sp.spheres_from_tensors(torch.from_numpy(cr).to("cuda:0"), torch.from_numpy(col).to("cuda:0"))
    torch.cuda.synchronize()
    return s, src, dst, cr, col


def r_unit_of(src):
    # the footprint of one source pixel at unit depth
    return 2.0 * src.tan_half_fov_y / src.height


@pytest.mark.parametrize("half_out", [True, False])
def test_codec_bit_exact_on_the_client_frame(sp, client, half_out):
    s, src, _, cr, k16 = client
    ru = r_unit_of(src)
    n = s.n()
    assert n == cr.shape[0]
    print(f"codec encode/decode {n} spheres, half out {half_out}", flush=True)
    pos, col = sp.encode_samples(s, LO, SIZE, ru)
    opos, ocol = oracle.encode(cr, k16.astype(np.float64), LO, SIZE, ru)
    gpos = pos[:n].cpu().numpy().view(np.uint64)
    gcol = col[:n].cpu().numpy().view(np.uint32)
    assert np.array_equal(gpos, opos), f"{(gpos != opos).sum()} position words differ"
    assert np.array_equal(gcol, ocol), f"{(gcol != ocol).sum()} colour words differ"
    d = sp.decode_samples(pos, col, s.count, LO, SIZE, ru, half=half_out)
    torch.cuda.synchronize()
    assert d.n() == n
    dcr, dcol = oracle.decode(opos, ocol, LO, SIZE, ru)
    g = d.centre_radius[:n].cpu().numpy()
    assert np.array_equal(g[:, :3], dcr[:, :3])
    # the radius goes through exp2: within one float ulp of the oracle's
    ulp = np.abs(g[:, 3].view(np.int32).astype(np.int64) - dcr[:, 3].view(np.int32))
    assert ulp.max() <= 1
    if half_out:
        b = np.stack([(ocol >> (8 * ch)) & 0xFF for ch in range(4)], axis=1).astype(np.float64) / 255.0
        # double -> half with round to nearest even (numpy's conversion; the
        # oracle's half rounding is pinned against it)
        assert np.array_equal(d.rgba[:n].cpu().numpy().view(np.uint16), b.astype(np.float16).view(np.uint16))
    else:
        assert np.array_equal(d.rgba[:n].cpu().numpy(), dcol)


def test_client_path_on_decoded_samples(sp, client):
    """Decoded spheres traced on the GPU match the oracle on the same decoded
    spheres; the image stays close to the one from the unquantised spheres."""
    s, src, dst, cr, k16 = client
    ru = r_unit_of(src)
    pos, col = sp.encode_samples(s, LO, SIZE, ru)
    d = sp.decode_samples(pos, col, s.count, LO, SIZE, ru, half=True)
    bvh = sp.build_bvh(d)
    img, hits = sp.trace(bvh, d, dst)
    ref_img, _ = sp.trace(sp.build_bvh(s), s, dst)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    pix = rng.integers(0, dst.width * dst.height, 2000)
    # the oracle's side: its own encode and decode of its own spheres (decoded
    # colours rounded to half, as the GPU stores them)
    opos, ocol = oracle.encode(cr, k16.astype(np.float64), LO, SIZE, ru)
    dcr, _ = oracle.decode(opos, ocol, LO, SIZE, ru)
    b = np.stack([(ocol >> (8 * ch)) & 0xFF for ch in range(4)], axis=1).astype(np.float64) / 255.0
    dcol = b.astype(np.float16)  # double -> half, round to nearest even
    g = img.cpu().numpy().reshape(-1, 4)[pix]
    h = hits.cpu().numpy().reshape(-1)[pix]
    assert_parity(compare(g, h, oracle.render(dcr, dcol, dst, pixels=pix)), exempt_frac=1e-4, context="decoded")
    diff = (img - ref_img).abs().mean().item()
    assert diff < 0.01, f"mean image change from the codec {diff}"


def test_codec_rejects_bad_parameters(sp, client):
    s, src = client[0], client[1]
    with pytest.raises(sp.SplatError):
        sp.encode_samples(s, LO, 0.0, 1e-3)
    with pytest.raises(sp.SplatError):
        sp.encode_samples(s, LO, SIZE, -1.0)


@pytest.mark.parametrize("half_out", [True, False])
def test_build_from_samples_equals_decode_then_build(sp, client, half_out):
    """The build that decodes the wire samples in its first kernel: the same
    spheres, count and BVH bytes as decode followed by build, and the same image."""
    s, src, dst, cr, k16 = client
    ru = r_unit_of(src)
    pos, col = sp.encode_samples(s, LO, SIZE, ru)
    print(f"build from samples half={half_out}", flush=True)
    d = sp.decode_samples(pos, col, s.count, LO, SIZE, ru, half=half_out)
    bvh = sp.build_bvh(d)
    f, fbvh = sp.build_bvh_from_samples(pos, col, s.count, LO, SIZE, ru, half=half_out)
    torch.cuda.synchronize()
    n = d.n()
    assert f.n() == n == s.n()
    assert torch.equal(f.centre_radius[:n], d.centre_radius[:n])
    assert torch.equal(f.rgba[:n].view(torch.int16) if half_out else f.rgba[:n], d.rgba[:n].view(torch.int16)
                       if half_out else d.rgba[:n])
    assert torch.equal(bvh_core(fbvh.mem, fbvh.capacity), bvh_core(bvh.mem, bvh.capacity)), "hierarchies differ"
    w0 = bvh_layout(bvh.capacity)["wide"]
    w1 = w0 + max(n - 1, 1) * 128
    assert torch.equal(fbvh.mem[w0:w1], bvh.mem[w0:w1]), "wide nodes differ"
    a, ha = sp.trace(bvh, d, dst)
    b, hb = sp.trace(fbvh, f, dst)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(ha, hb)
    # a count below the capacity: only that many samples are decoded
    few = torch.tensor([1000], dtype=torch.int32, device="cuda:0")
    g, gbvh = sp.build_bvh_from_samples(pos, col, few, LO, SIZE, ru, half=half_out)
    torch.cuda.synchronize()
    assert g.n() == 1000 and torch.equal(g.centre_radius[:1000], d.centre_radius[:1000])
    assert gbvh.status() == 0
