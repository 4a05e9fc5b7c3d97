"""GPU parity of the sample codec (splat_encode_samples / splat_decode_samples,
the wire format of Sec. 4.1 and Sec. 5) against the oracle's codec, and the
client path run on decoded samples."""
import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import assert_parity, compare

pytestmark = pytest.mark.gpu
LO, SIZE = synth.BOX_LO, synth.BOX_SIZE


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


@pytest.fixture(scope="module")
def client(sp):
    rgba, depth, src, dst = synth.source_image(synth.CLIENT_FRAME)
    s = sp.unproject(src, torch.from_numpy(rgba).to("cuda:0"), torch.from_numpy(depth).to("cuda:0"), 1.0, True)
    torch.cuda.synchronize()
    return s, src, dst


def r_unit_of(src):
    # the footprint of one source pixel at unit depth
    return 2.0 * src.tan_half_fov_y / src.height


@pytest.mark.parametrize("half_out", [True, False])
def test_codec_bit_exact_on_the_client_frame(sp, client, half_out):
    s, src, _ = client
    ru = r_unit_of(src)
    n = s.n()
    print(f"codec encode/decode {n} spheres, half out {half_out}", flush=True)
    pos, col = sp.encode_samples(s, LO, SIZE, ru)
    cr = s.centre_radius[:n].cpu().numpy()
    k = s.rgba[:n].cpu().numpy().astype(np.float64)
    opos, ocol = oracle.encode(cr, k, LO, SIZE, ru)
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
    s, src, dst = client
    ru = r_unit_of(src)
    n = s.n()
    pos, col = sp.encode_samples(s, LO, SIZE, ru)
    d = sp.decode_samples(pos, col, s.count, LO, SIZE, ru, half=True)
    bvh = sp.build_bvh(d)
    img, hits = sp.trace(bvh, d, dst)
    ref_img, _ = sp.trace(sp.build_bvh(s), s, dst)
    torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    pix = rng.integers(0, dst.width * dst.height, 2000)
    dcr = d.centre_radius[:n].cpu().numpy()
    dcol = d.rgba[:n].cpu().numpy()
    g = img.cpu().numpy().reshape(-1, 4)[pix]
    h = hits.cpu().numpy().reshape(-1)[pix]
    assert_parity(compare(g, h, oracle.render(dcr, dcol, dst, pixels=pix)), exempt_frac=1e-4, context="decoded")
    diff = (img - ref_img).abs().mean().item()
    assert diff < 0.01, f"mean image change from the codec {diff}"


def test_codec_rejects_bad_parameters(sp, client):
    s, src, _ = client
    with pytest.raises(sp.SplatError):
        sp.encode_samples(s, LO, 0.0, 1e-3)
    with pytest.raises(sp.SplatError):
        sp.encode_samples(s, LO, SIZE, -1.0)
