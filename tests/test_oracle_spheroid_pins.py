"""Pins of the oracle's spheroids: samples smeared along their source ray over
their depth interval (Sec. 7 suggests it; the shape is this library's
reading: a prolate spheroid with its long axis on the source ray).
* closed forms with the ray along the axis (entry at the tip), across it
  (entry at the lateral radius), off-centre and tangent;
* the spheroid with h = r is the sphere of the sphere test, and its render
  is the sphere render;
* the robust form equals the smaller root of the textbook world-space
  quadratic (numpy.roots) on random non-grazing cases, is unchanged by a
  rigid motion of the scene and by flipping the axis;
* the unprojection: centre on the pixel ray at the interval's midpoint,
  radius the footprint there, axis the unit pixel ray, half-length
  max(r, kappa half-interval), hand-computed on the optical axis;
* a view along the source ray sees the spheroid's tip first."""
import math

import numpy as np
import pytest

import oracle
import synth
from test_oracle_policy_pins import _one_pixel

O = np.zeros(3)
Z = np.array([0.0, 0.0, 1.0])


@pytest.mark.parametrize("c,u,t0,disc", [((0, 0, 5), (0, 0, 1), 3.0, 1.0),       # along the axis: the tip at 5 - h
                                         ((0, 0, 5), (1, 0, 0), 4.5, 1.0),       # across it: 5 - r
                                         ((1, 0, 5), (1, 0, 0), 5.0 - math.sqrt(0.1875), 0.75),
                                         ((2, 0, 5), (1, 0, 0), 5.0, 0.0),       # tangent at the tip
                                         ((0, 0.5, 5), (1, 0, 0), 5.0, 0.0)])    # tangent at the side
def test_spheroid_closed_form(c, u, t0, disc):
    hit, t, dsc, tm, qq = oracle.spheroid_test(O, Z, c, 0.5, u, 2.0)
    assert hit
    assert t == pytest.approx(t0, abs=1e-12)
    assert dsc == pytest.approx(disc, abs=1e-12)
    assert qq == pytest.approx(1.0 - disc, abs=1e-12)


def test_spheroid_misses_and_eye_inside():
    assert not oracle.spheroid_test(O, Z, (2.01, 0, 5), 0.5, (1, 0, 0), 2.0)[0]   # beyond the tip
    assert not oracle.spheroid_test(O, Z, (0, 0.51, 5), 0.5, (1, 0, 0), 2.0)[0]   # beyond the side
    assert not oracle.spheroid_test(O, Z, (0, 0, -5), 0.5, (0, 0, 1), 2.0)[0]     # behind the eye
    assert not oracle.spheroid_test(O, Z, (0, 0, 1), 0.5, (0, 0, 1), 2.0)[0]      # the eye inside: entry < 0
    assert not oracle.spheroid_test(O, Z, (0, 0, 5), 0.5, (0, 0, 1), 2.0, t_max=3.0)[0]


def test_equal_half_length_is_the_sphere():
    rng = np.random.default_rng(3)
    for _ in range(200):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = rng.uniform(0.05, 1.0)
        c = d * rng.uniform(2, 6) + rng.normal(size=3) * r * 0.7
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        hs, ts, qs, ds, _, _ = oracle.sphere_test(O, d, c, r)
        he, te, de, _, _ = oracle.spheroid_test(O, d, c, r, u, r)
        assert hs == he
        assert de == pytest.approx(ds / (r * r), abs=1e-12)
        if hs:
            assert te == pytest.approx(ts, rel=1e-12)


def _quadratic_t0(o, d, c, r, u, h):
    """Smaller root of the world-space quadratic |P(x - c)|^2 / r^2 + ((x - c).u)^2 / h^2 = 1 on x = o + t d."""
    w = np.asarray(o, float) - np.asarray(c, float)
    k = 1.0 / h ** 2 - 1.0 / r ** 2
    du, wu = float(np.dot(d, u)), float(np.dot(w, u))
    A = np.dot(d, d) / r ** 2 + du * du * k
    B = 2.0 * (np.dot(w, d) / r ** 2 + wu * du * k)
    C = np.dot(w, w) / r ** 2 + wu * wu * k - 1.0
    roots = np.roots([A, B, C])
    if np.any(np.abs(roots.imag) > 0):
        return None
    return float(np.min(roots.real))


def test_spheroid_matches_quadratic_roots():
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(400):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = rng.uniform(0.05, 0.5)
        h = r * rng.uniform(1.0, 8.0)
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        c = d * rng.uniform(3, 8) + rng.normal(size=3) * h * 0.6
        hit, t0, disc, _, _ = oracle.spheroid_test(O, d, c, r, u, h)
        want = _quadratic_t0(O, d, c, r, u, h)
        if abs(disc) < 1e-6:
            continue
        assert hit == (want is not None and want > 0)
        if hit:
            assert t0 == pytest.approx(want, rel=1e-9)
            checked += 1
    assert checked > 100


def test_rigid_motion_and_axis_flip_leave_the_entry_unchanged():
    rng = np.random.default_rng(9)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    shift = rng.normal(size=3)
    hits = 0
    for _ in range(100):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r, h = 0.3, 1.1
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        c = d * 4.0 + rng.normal(size=3) * 0.5
        a = oracle.spheroid_test(O, d, c, r, u, h)
        b = oracle.spheroid_test(shift, q @ d, q @ c + shift, r, q @ u, h)
        f = oracle.spheroid_test(O, d, c, r, -u, h)
        assert a[0] == b[0] == f[0]  # hit or miss alike
        assert a[2] == pytest.approx(b[2], abs=1e-12) and a[2] == pytest.approx(f[2], abs=1e-12)
        if a[2] >= 0:
            hits += 1
            assert a[1] == pytest.approx(b[1], rel=1e-12) and a[1] == pytest.approx(f[1], rel=1e-12)
    assert hits > 20


def test_spheroids_with_equal_half_length_render_as_spheres():
    cr, col = synth.random_spheres(150, seed=4, r_lo=0.03, r_hi=0.1)
    cam = synth.rotated_camera(synth.source_camera(40, 30), 7.0, 2.0)
    rng = np.random.default_rng(2)
    u = rng.normal(size=(cr.shape[0], 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    axis = np.concatenate([u, cr[:, 3:4].astype(np.float64)], axis=1).astype(np.float32)
    a = oracle.render(cr, col, cam)
    b = oracle.render(cr, col, cam, axis=axis)
    assert np.array_equal(a["n"], b["n"]) and np.array_equal(a["sig"], b["sig"])
    assert np.allclose(a["rgba"], b["rgba"], atol=1e-12, rtol=0)
    assert int(a["n"].sum()) > 300


def test_unproject_spheroids_on_the_axis_hand_computed():
    # interval [1, 3] on the optical axis of the 3x3 view from (0, 0, 5): centre at t = 2, footprint 2/3
    cam, rgba, depth, itv = _one_pixel(A=0.25, t=1.7, interval=(1.0, 3.0))
    for kappa, h in [(0.25, 1.0), (2.0, 2.0), (1.0, 1.0), (0.5, 1.0)]:
        cr, col, idx, ax = oracle.unproject_spheroids(cam, rgba, depth, itv, radius_scale=1.5, interval_scale=kappa)
        assert idx.tolist() == [4]
        assert cr[0].tolist() == [0.0, 0.0, 3.0, 1.0], kappa      # r = 1.5 (2/3), the footprint at t_c
        assert ax[0].tolist() == [0.0, 0.0, -1.0, h], kappa       # axis: the source ray; h = max(r, kappa 1)
        assert col[0].astype(np.float64).tolist() == [0.5, 0.25, 1.0, 0.25]
    # invalid intervals drop the pixel, as in the interval policy
    cam, rgba, depth, itv = _one_pixel(A=0.5, t=2.0, interval=(3.0, 1.0))
    assert oracle.unproject_spheroids(cam, rgba, depth, itv)[0].shape[0] == 0


def test_unproject_spheroids_lie_along_the_pixel_rays():
    rgba, depth, src, _ = synth.source_image(synth.TINY)
    vol = synth.volume_of(synth.TINY)
    m = oracle.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src)
    itv = m["interval"].astype(np.float32).reshape(src.height, src.width, 2)
    cr, _, idx, ax = oracle.unproject_spheroids(src, rgba, depth, itv, interval_scale=1.0)
    ci, _, idx_i = oracle.unproject_policy(src, rgba, depth, oracle.RADIUS_INTERVAL, interval_scale=1.0,
                                           interval=itv)
    assert np.array_equal(idx, idx_i) and idx.size > 400
    assert np.array_equal(cr[:, :3], ci[:, :3])   # the same centres as the interval policy
    eye = np.array(src.eye)
    lo, hi = itv.reshape(-1, 2)[idx].astype(np.float64).T
    off = cr[:, :3].astype(np.float64) - eye
    u = ax[:, :3].astype(np.float64)
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-6)
    # the axis points along the centre's offset from the eye (the pixel ray), to float rounding
    cos = np.sum(off * u, axis=1) / (np.linalg.norm(off, axis=1) * np.linalg.norm(u, axis=1))
    assert np.all(cos > 1 - 1e-12)
    # r is the footprint at the midpoint; h covers the interval at kappa = 1 and is never below r
    fp = 2.0 * 0.5 * (lo + hi) * src.tan_half_fov_y / src.height
    assert np.allclose(cr[:, 3].astype(np.float64), fp, rtol=1e-6)
    h = ax[:, 3].astype(np.float64)
    assert np.all(h >= cr[:, 3] * (1 - 1e-7))
    assert np.allclose(h, np.maximum(fp, 0.5 * (hi - lo)), rtol=1e-6)


def test_view_along_the_source_ray_meets_the_tip():
    """Seen from its own source camera the spheroid's axis is the pixel ray: the entry is at t_c - h."""
    cam, rgba, depth, itv = _one_pixel(A=0.75, t=2.0, interval=(1.0, 3.0))
    cr, col, idx, ax = oracle.unproject_spheroids(cam, rgba, depth, itv, radius_scale=0.1, interval_scale=1.0)
    hit, t0, disc, _, _ = oracle.spheroid_test(np.array(cam.eye), np.array(cam.forward), cr[0, :3].astype(np.float64),
                                               float(cr[0, 3]), ax[0, :3].astype(np.float64), float(ax[0, 3]))
    assert hit and t0 == pytest.approx(1.0, abs=1e-7) and disc == pytest.approx(1.0, abs=1e-6)
    orc = oracle.render(cr, col, cam, pixels=[4], axis=ax)
    assert orc["n"][0] == 1 and orc["rgba"][0][3] == pytest.approx(0.75)


def test_spheroid_tangent_pixel_is_flagged_grazing():
    """The optical-axis pixel of the 3x3 view touches the tip of a spheroid lying across the view: exempt."""
    cam, _, _, _ = _one_pixel()
    cr = np.array([[0.5, 0.0, 2.0, 0.25], [0.0, 0.3, 1.0, 0.25]], dtype=np.float32)
    col = np.array([[1, 0, 0, 0.5], [0, 1, 0, 0.5]], dtype=np.float32)
    ax = np.array([[1.0, 0.0, 0.0, 0.5], [0.0, 0.0, 1.0, 0.25]], dtype=np.float32)
    orc = oracle.render(cr, col, cam, axis=ax)
    assert orc["flags"][4] & oracle.FLAG_GRAZE
    assert orc["n"][4] == 1 and orc["rgba"][4][0] == pytest.approx(0.5)
    # a sphere of the lateral radius would not even be near: the shape, not its bounding sphere, decides
    assert not (oracle.render(cr, col, cam)["flags"][4] & oracle.FLAG_GRAZE)
    # inside the band but not touching: disc = 1 - (2 x)^2 = 4.8e-7 of the unit ball (the band is 1e-6 of it)
    cr[0, 0] = np.float32(0.5 - 1.25e-7)
    hit, _, disc, _, _ = oracle.spheroid_test(cam.eye, cam.forward, cr[0, :3].astype(np.float64), 0.25,
                                              ax[0, :3].astype(np.float64), 0.5)
    assert hit and 1e-7 < disc < 1e-6
    assert oracle.render(cr, col, cam, axis=ax)["flags"][4] & oracle.FLAG_GRAZE
