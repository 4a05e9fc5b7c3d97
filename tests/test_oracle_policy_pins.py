"""Pins of the oracle's radius policies (Sec. 7: the radius varied with the
sample's opacity, or the sample smeared over a depth interval along the ray;
the rules are this library's readings) and of the marcher's depth interval:
* the interval through a constant volume from the closed form 1 - (1 - s)^k,
  including an interval that never reaches its upper alpha and one cut by
  the stop;
* hand-computed centres and radii on a ray along the optical axis, the
  floor, and the invalid intervals that drop a pixel;
* geometry that holds off-axis: the interval centre lies on the pixel's ray
  at the interval's midpoint;
* the footprint policy is the plain unprojection, and the opacity policy at
  full opacity is the footprint policy."""
import math

import numpy as np
import pytest

import oracle
import synth
from test_oracle_march_pins import _axis_camera


def _interval_closed_form(value, t_in, t_out, n, size, lo_a=0.25, hi_a=0.75, stop=0.999, alpha_scale=0.05):
    s = min(max(alpha_scale * value, 0.0), 1.0)
    dt = 0.5 * size / n
    k_in = max(0, math.ceil((t_out - t_in) / dt - 0.5))
    k_stop = math.ceil(math.log(1.0 - stop) / math.log(1.0 - s))
    k = min(k_in, k_stop)  # samples taken

    def first(alpha):
        return math.ceil(math.log(1.0 - alpha) / math.log(1.0 - s))

    t_of = lambda j: t_in + (j - 0.5) * dt  # noqa: E731  (j counted from 1)
    k_lo, k_hi = first(lo_a), first(hi_a)
    if k_lo > k:
        return math.inf, math.inf
    return t_of(k_lo), t_of(k_hi if k_hi <= k else k)


@pytest.mark.parametrize("value,stop", [(12.0, 0.999), (1.7, 0.999), (0.6, 0.999), (0.3, 0.999), (1.7, 0.5),
                                        (0.05, 0.999)])
def test_marcher_interval_closed_form(value, stop):
    n, lo, size = 32, -0.25, 1.5
    vol = np.full((n, n, n), value, dtype=np.float32)
    centre = lo + size / 2
    cam = _axis_camera(5, 5, (centre, centre, 3.0), (0.0, 0.0, -1.0))
    got = oracle.raymarch(vol, lo, size, cam, pixels=[12], stop_alpha=stop)
    v32 = float(np.float32(value))
    want = _interval_closed_form(v32, 3.0 - (lo + size), 3.0 - lo, n, size, stop=stop)
    for g, w in zip(got["interval"][0], want):
        if math.isinf(w):
            assert math.isinf(g)
        else:
            assert g == pytest.approx(w, rel=1e-12)
    if value == 0.3:  # A stays below 0.75: the interval closes at the last sample
        assert want[1] == pytest.approx(3.0 - lo - 0.5 * 0.5 * size / n)
    if value == 0.05:  # A never reaches 0.25
        assert math.isinf(want[0])
    lo_t, hi_t, d = got["interval"][0][0], got["interval"][0][1], got["depth"][0]
    if math.isfinite(d):
        assert lo_t <= d <= hi_t


def _one_pixel(A=0.25, t=2.0, interval=None):
    """A 3x3 source view down -z from (0, 0, 5), tan(fov/2) = 0.5; only the
    centre pixel, whose ray is the optical axis, holds a sample."""
    cam = synth.Camera((0.0, 0.0, 5.0), (0.0, 0.0, -1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.5, 3, 3)
    rgba = np.zeros((3, 3, 4), dtype=np.float32)
    rgba[1, 1] = (0.5 * A, 0.25 * A, 1.0 * A, A)
    depth = np.full((3, 3), np.inf, dtype=np.float32)
    depth[1, 1] = t
    itv = np.full((3, 3, 2), np.inf, dtype=np.float32)
    if interval is not None:
        itv[1, 1] = interval
    return cam, rgba, depth, itv


def test_policies_on_the_axis_hand_computed():
    # footprint at t = 2: 2 t tan / H = 2/3
    cam, rgba, depth, itv = _one_pixel(A=0.25)
    cr, col, idx = oracle.unproject_policy(cam, rgba, depth, oracle.RADIUS_FOOTPRINT, radius_scale=1.5)
    assert idx.tolist() == [4] and cr[0].tolist() == [0.0, 0.0, 3.0, 1.0]
    cr, _, _ = oracle.unproject_policy(cam, rgba, depth, oracle.RADIUS_OPACITY, radius_scale=1.5)
    assert cr[0].tolist() == [0.0, 0.0, 3.0, 0.5]  # 1.5 (2/3) sqrt(0.25)
    cam, rgba, depth, itv = _one_pixel(A=0.01)
    cr, _, _ = oracle.unproject_policy(cam, rgba, depth, oracle.RADIUS_OPACITY, radius_scale=1.5, opacity_floor=0.04)
    assert cr[0, 3] == pytest.approx(0.2, rel=1e-6)  # the floor: 1.5 (2/3) sqrt(0.04)
    # interval [1, 3]: centre at t = 2, half length 1
    cam, rgba, depth, itv = _one_pixel(A=0.25, t=1.7, interval=(1.0, 3.0))
    for kappa, r in [(0.25, 1.0), (2.0, 2.0), (0.0, 1.0)]:
        cr, col, idx = oracle.unproject_policy(cam, rgba, depth, oracle.RADIUS_INTERVAL, radius_scale=1.5,
                                               interval_scale=kappa, interval=itv)
        assert cr[0].tolist() == [0.0, 0.0, 3.0, r], kappa
    # the colour is the plain unprojection's in every policy: straight, alpha A
    assert col[0].astype(np.float64).tolist() == [0.5, 0.25, 1.0, 0.25]


@pytest.mark.parametrize("bad", [(np.inf, 3.0), (1.0, np.inf), (3.0, 1.0), (0.0, 1.0), (-1.0, 1.0), (np.nan, 1.0)])
def test_invalid_interval_drops_the_pixel(bad):
    cam, rgba, depth, itv = _one_pixel(A=0.5, t=2.0, interval=bad)
    cr, _, _ = oracle.unproject_policy(cam, rgba, depth, oracle.RADIUS_INTERVAL, interval=itv)
    assert cr.shape[0] == 0
    # the other policies ignore the interval
    cr, _, _ = oracle.unproject_policy(cam, rgba, depth, oracle.RADIUS_OPACITY, interval=itv)
    assert cr.shape[0] == 1


def test_interval_centre_on_the_pixel_ray():
    rgba, depth, src, _ = synth.source_image(synth.TINY)
    vol = synth.volume_of(synth.TINY)
    m = oracle.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src)
    itv = m["interval"].astype(np.float32).reshape(src.height, src.width, 2)
    cr0, _, idx0 = oracle.unproject_policy(src, rgba, depth, oracle.RADIUS_FOOTPRINT)
    cr2, _, idx2 = oracle.unproject_policy(src, rgba, depth, oracle.RADIUS_INTERVAL, interval_scale=1.0, interval=itv)
    assert idx2.size > 400 and set(idx2.tolist()) <= set(idx0.tolist())
    where = {int(p): j for j, p in enumerate(idx0)}
    eye = np.array(src.eye)
    lo, hi = itv.reshape(-1, 2)[idx2].astype(np.float64).T
    a = cr2[:, :3].astype(np.float64) - eye
    b = cr0[[where[int(p)] for p in idx2], :3].astype(np.float64) - eye
    # distance from the eye: the midpoint; direction: that of the plain sample (same pixel ray)
    assert np.allclose(np.linalg.norm(a, axis=1), 0.5 * (lo + hi), rtol=1e-6)
    cos = np.sum(a * b, axis=1) / (np.linalg.norm(a, axis=1) * np.linalg.norm(b, axis=1))
    assert np.all(cos > 1 - 1e-9)
    # the sphere covers the interval at kappa = 1
    assert np.all(cr2[:, 3].astype(np.float64) >= 0.5 * (hi - lo) * (1 - 1e-6))


def test_footprint_policy_is_the_plain_unprojection_and_full_opacity_too():
    rgba, depth, src, _ = synth.source_image(synth.TINY)
    for half in (True, False):
        a = oracle.unproject(src, rgba, depth, 1.25, half)
        b = oracle.unproject_policy(src, rgba, depth, oracle.RADIUS_FOOTPRINT, radius_scale=1.25, half=half)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    opaque = rgba.copy()
    opaque[..., :3] /= np.maximum(opaque[..., 3:], 1e-30)
    opaque[..., 3] = np.where(rgba[..., 3] > 0, 1.0, 0.0)
    f = oracle.unproject_policy(src, opaque, depth, oracle.RADIUS_FOOTPRINT)
    o = oracle.unproject_policy(src, opaque, depth, oracle.RADIUS_OPACITY)
    assert np.array_equal(f[0], o[0])
    # and the opacity radius grows with the opacity
    o2 = oracle.unproject_policy(src, rgba, depth, oracle.RADIUS_OPACITY, opacity_floor=1e-6)
    A = rgba.reshape(-1, 4)[o2[2], 3].astype(np.float64)
    ratio = o2[0][:, 3].astype(np.float64) / f[0][:, 3].astype(np.float64)
    assert np.allclose(ratio, np.sqrt(A), rtol=1e-6)
