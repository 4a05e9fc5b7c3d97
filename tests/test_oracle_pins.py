"""Pins of the FP64 oracle against closed forms, hand-computed composites,
library routines and invariants.  CPU only.

Each test names the part of the paper (or the reading of it) that it pins.
"""
import math

import numpy as np
import pytest

import oracle
import synth


class Cam:
    """Minimal camera record (the oracle reads attributes only)."""

    def __init__(self, eye, forward, right, up, tan_half_fov_y, width, height):
        self.eye, self.forward, self.right, self.up = eye, forward, right, up
        self.tan_half_fov_y, self.width, self.height = tan_half_fov_y, width, height


# A 1x1 camera at the origin looking along +z: its only ray is o = 0, d = +z.
AXIS_CAM = Cam((0.0, 0.0, 0.0), (0.0, 0.0, 1.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 0.5, 1, 1)
NEVER = 2.0  # alpha_stop above 1: composite every hit


def table(rows):
    """rows of (cx, cy, cz, r, kr, kg, kb, a)."""
    return np.array(rows, dtype=np.float64)


# ------------------------------------------------------------ ray-sphere (hit rule)

@pytest.mark.parametrize("c,r,hit,t0,q", [
    ((0, 0, 5), 1.0, True, 4.0, 0.0),
    ((0.6, 0, 5), 1.0, True, 4.2, 0.36),
    ((1, 0, 5), 1.0, True, 5.0, 1.0),      # tangent: disc = 0 counts as a hit
    ((0, 0, -5), 1.0, False, None, 0.0),   # behind the eye
    ((0, 0, 0.5), 1.0, False, None, 0.0),  # eye inside: t0 < 0, skipped
    ((2, 0, 5), 1.0, False, None, 4.0),    # clean miss
])
def test_sphere_closed_form(c, r, hit, t0, q):
    h, tt, qq, disc, v, b = oracle.sphere_test((0, 0, 0), (0, 0, 1), c, r)
    assert h == hit
    assert qq == pytest.approx(q, abs=1e-15)
    assert disc == pytest.approx(r * r - q, abs=1e-15)
    if t0 is not None:
        assert tt == pytest.approx(t0, abs=1e-15)
    assert b == pytest.approx(c[2], abs=1e-15)
    assert np.allclose(v, (c[0], c[1], 0.0), atol=1e-15)


def test_sphere_t_max_bounds_the_hit():
    assert oracle.sphere_test((0, 0, 0), (0, 0, 1), (0, 0, 5), 1.0, t_max=4.5)[0]
    assert not oracle.sphere_test((0, 0, 0), (0, 0, 1), (0, 0, 5), 1.0, t_max=4.0)[0]


def test_sphere_matches_quadratic_roots():
    """|o + t d - c|^2 = r^2 solved by numpy.roots agrees with the robust form (off-axis rays)."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        c = rng.uniform(-3, 3, size=3) + 4 * d
        r = rng.uniform(0.1, 2.0)
        oc = c
        roots = np.roots([1.0, -2.0 * np.dot(d, oc), np.dot(oc, oc) - r * r])
        real = np.sort(roots[np.abs(roots.imag) < 1e-12].real)
        hit, t0, q, disc, v, b = oracle.sphere_test((0, 0, 0), d, c, r)
        if abs(disc) < 1e-9:
            continue
        if disc > 0:
            assert real.size == 2
            assert t0 == pytest.approx(real[0], rel=1e-9, abs=1e-9)
            assert hit == (real[0] > 0)
        else:
            assert not hit


# ------------------------------------------------------------ compositing (front to back)

def test_two_spheres_hand_computed():
    red = (0, 0, 5, 1, 1, 0, 0, 0.5)      # t0 = 4
    green = (0, 0, 5.5, 1, 0, 1, 0, 0.5)  # t0 = 4.5
    out = oracle.render_table(table([red, green]), AXIS_CAM, alpha_stop=NEVER)
    assert np.allclose(out["rgba"][0], (0.5, 0.25, 0.0, 0.75), atol=1e-15)
    assert out["n"][0] == 2
    # swapping the depths swaps the weights: order matters
    red2 = (0, 0, 5.5, 1, 1, 0, 0, 0.5)
    green2 = (0, 0, 5, 1, 0, 1, 0, 0.5)
    out = oracle.render_table(table([red2, green2]), AXIS_CAM, alpha_stop=NEVER)
    assert np.allclose(out["rgba"][0], (0.25, 0.5, 0.0, 0.75), atol=1e-15)


def four():
    return table([(0, 0, 5.0, 1, 1, 0, 0, 0.8), (0, 0, 5.5, 1, 0, 1, 0, 0.8),
                  (0, 0, 6.0, 1, 0, 0, 1, 0.8), (0, 0, 6.5, 1, 1, 1, 1, 0.8)])


def test_stop_at_alpha_hand_computed():
    out = oracle.render_table(four(), AXIS_CAM, alpha_stop=0.99)
    assert np.allclose(out["rgba"][0], (0.8, 0.16, 0.032, 0.992), atol=1e-15)
    assert out["n"][0] == 3
    out = oracle.render_table(four(), AXIS_CAM, alpha_stop=NEVER)
    assert np.allclose(out["rgba"][0], (0.8064, 0.1664, 0.0384, 0.9984), atol=1e-15)
    assert out["n"][0] == 4


def test_first_hit_special_case():
    """alpha_stop = 0: the paper's first-hit query returns a k of the nearest sphere."""
    out = oracle.render_table(four()[::-1].copy(), AXIS_CAM, alpha_stop=0.0)
    assert np.allclose(out["rgba"][0], (0.8, 0.0, 0.0, 0.8), atol=1e-15)
    assert out["n"][0] == 1


def test_equal_depth_tie_breaks_by_id():
    a = (0, 0, 5, 1, 1, 0, 0, 0.5)
    b = (0, 0, 5, 1, 0, 1, 0, 0.5)
    out = oracle.render_table(table([a, b]), AXIS_CAM, alpha_stop=NEVER)
    assert np.allclose(out["rgba"][0], (0.5, 0.25, 0, 0.75), atol=1e-15)  # id 0 first
    out = oracle.render_table(table([b, a]), AXIS_CAM, alpha_stop=NEVER)
    assert np.allclose(out["rgba"][0], (0.25, 0.5, 0, 0.75), atol=1e-15)


def test_stop_knife_edge_reports_both_branches():
    a = (0, 0, 5, 1, 1, 0, 0, 0.5)
    b = (0, 0, 5.5, 1, 0, 1, 0, 0.5)
    c = (0, 0, 6.0, 1, 0, 0, 1, 0.5)
    out = oracle.render_table(table([a, b, c]), AXIS_CAM, alpha_stop=0.75)  # A = 0.75 exactly after 2
    assert out["flags"][0] & oracle.FLAG_KNIFE
    assert out["n"][0] == 2 and out["alt_n"][0] == 3
    assert np.allclose(out["alt_rgba"][0], (0.5, 0.25, 0.125, 0.875), atol=1e-15)


def test_tangent_sphere_is_flagged_grazing():
    out = oracle.render_table(table([(1, 0, 5, 1, 1, 1, 1, 0.5)]), AXIS_CAM, alpha_stop=NEVER)
    assert out["flags"][0] & oracle.FLAG_GRAZE
    out = oracle.render_table(table([(0.5, 0, 5, 1, 1, 1, 1, 0.5)]), AXIS_CAM, alpha_stop=NEVER)
    assert out["flags"][0] == 0


def test_hit_sets_against_quadratic_roots_on_tiny_scene():
    """Hit count and final alpha 1 - prod(1 - a_i) (order-free) against numpy.roots per ray and sphere."""
    cr, col = synth.random_spheres(60, seed=5, r_lo=0.05, r_hi=0.2)
    cam = synth.rotated_camera(synth.source_camera(12, 10), 7.0, 2.0)
    out = oracle.render(cr, col, cam, alpha_stop=NEVER)
    tab = oracle.sphere_table(cr, col)
    eye = np.array(cam.eye)
    F, R, U = (np.array(v) for v in (cam.forward, cam.right, cam.up))
    checked = 0
    for p in range(cam.width * cam.height):
        if out["flags"][p]:
            continue
        x, y = p % cam.width, p // cam.width
        # ray through the pixel centre, written as a point on the image plane at distance 1
        px = ((x + 0.5) / cam.width * 2 - 1) * cam.tan_half_fov_y * cam.width / cam.height
        py = (1 - (y + 0.5) / cam.height * 2) * cam.tan_half_fov_y
        target = eye + F + px * R + py * U
        d = (target - eye) / np.linalg.norm(target - eye)
        trans, nh = 1.0, 0
        for s in tab:
            oc = s[:3] - eye
            roots = np.roots([1.0, -2.0 * np.dot(d, oc), np.dot(oc, oc) - s[3] ** 2])
            real = roots[np.abs(roots.imag) < 1e-12].real
            if real.size == 2 and min(real) > 0:
                nh += 1
                trans *= 1 - s[7]
        assert out["n"][p] == nh
        assert out["rgba"][p][3] == pytest.approx(1 - trans, abs=1e-12)
        checked += nh
    assert checked > 20


# ------------------------------------------------------------ unprojection (Eq. 1)

def test_unproject_eq1_closed_form():
    """2x2 image, fov 90 deg: pixel (0,0) looks along (-1/2, 1/2, -1)/sqrt(3/2); p = o + d t."""
    cam = Cam((0.25, -0.5, 3.0), (0, 0, -1), (1, 0, 0), (0, 1, 0), 1.0, 2, 2)
    rgba = np.zeros((2, 2, 4), dtype=np.float32)
    depth = np.full((2, 2), np.inf, dtype=np.float32)
    t = np.float32(math.sqrt(1.5))
    rgba[0, 0] = (0.25, 0.5, 0.125, 0.5)
    depth[0, 0] = t
    cr, colour, idx = oracle.unproject(cam, rgba, depth, radius_scale=2.0, half=False)
    assert idx.tolist() == [0]
    d = np.array([-0.5, 0.5, -1.0]) / math.sqrt(1.5)
    p = np.array(cam.eye) + d * float(t)
    assert np.array_equal(cr[0, :3], p.astype(np.float32))
    # radius = s * footprint = 2 * (2 t tan(45 deg) / H)
    assert cr[0, 3] == np.float32(2.0 * 2.0 * float(t) * 1.0 / 2.0)
    assert np.array_equal(colour[0], np.array([0.5, 1.0, 0.25, 0.5], dtype=np.float32))


def test_unproject_colour_is_straight_and_clamped():
    """k = clamp(C / A, 0, 1): a premultiplied value above A clamps to 1, a negative one to 0."""
    cam = Cam((0.0, 0.0, 3.0), (0, 0, -1), (1, 0, 0), (0, 1, 0), 1.0, 1, 1)
    rgba = np.array([[[0.75, -0.25, 0.2, 0.5]]], dtype=np.float32)
    depth = np.array([[2.0]], dtype=np.float32)
    _, colour, _ = oracle.unproject(cam, rgba, depth, 1.0, half=False)
    assert np.array_equal(colour[0], np.array([1.0, 0.0, np.float32(0.2 / 0.5), 0.5], dtype=np.float32))


def test_unproject_footprint_values():
    """At t = 2 with fov 45 deg: footprint 2 t tan(22.5 deg) / H."""
    for H, expect in [(64, 0.0258883476), (512, 0.00323604345), (1024, 0.00161802172)]:
        cam = synth.source_camera(1, H)
        rgba = np.zeros((H, 1, 4), dtype=np.float32)
        rgba[:, :, 3] = 0.5
        depth = np.full((H, 1), 2.0, dtype=np.float32)
        cr, _, _ = oracle.unproject(cam, rgba, depth, 1.0, half=False)
        assert cr[0, 3] == pytest.approx(expect, rel=1e-7)


def test_unproject_compaction_is_stable_and_filters_invalid():
    rng = np.random.default_rng(3)
    cam = synth.source_camera(17, 13)
    rgba = rng.uniform(0.1, 0.5, size=(13, 17, 4)).astype(np.float32)
    rgba[..., 3] = rng.uniform(0.5, 1.0, size=(13, 17))
    depth = rng.uniform(1.5, 2.5, size=(13, 17)).astype(np.float32)
    flat = depth.ravel()
    flat[::7] = np.inf
    flat[3::11] = np.nan
    flat[5::13] = 0.0
    flat[6::17] = -1.0
    rgba.reshape(-1, 4)[9::19, 3] = 0.0
    valid = np.isfinite(flat) & (flat > 0) & (rgba.reshape(-1, 4)[:, 3] > 0)
    cr, colour, idx = oracle.unproject(cam, rgba, depth, 1.0, half=True)
    assert np.array_equal(idx, np.nonzero(valid)[0].astype(np.uint32))
    assert colour.dtype == np.float16


def test_half_rounding_matches_numpy():
    rng = np.random.default_rng(0)
    v = np.concatenate([rng.uniform(0, 1, 4000), rng.uniform(0, 1e-4, 500),
                        [0.0, 1.0, 1 + 2 ** -11, 1 + 3 * 2 ** -11, 2 ** -24, 2 ** -25, 3 * 2 ** -25,
                         65504.0, 65519.0, 65520.0, 2 ** -14, 2 ** -14 - 2 ** -25, 0.1, 1 / 3]])
    ours = oracle.half_bits(v)
    ref = v.astype(np.float16).view(np.uint16)
    assert np.array_equal(ours, ref)


# ------------------------------------------------------------ invariants on generator inputs

def test_identity_reprojection_reproduces_source():
    """Target camera = source camera, radius scale 0.01: every pixel returns its premultiplied RGBA."""
    rgba, depth, src, _ = synth.source_image(synth.TINY)
    cr, colour, idx = oracle.unproject(src, rgba, depth, 0.01, half=False)
    out = oracle.render(cr, colour, src, alpha_stop=0.99)
    img = out["rgba"].reshape(src.height, src.width, 4)
    has = np.isfinite(depth) & (depth > 0)
    assert has.sum() == len(idx) > 100
    assert np.abs(img[has] - rgba[has]).max() <= 1e-6
    assert np.all(img[~has] == 0)
    assert np.all(out["n"].reshape(src.height, src.width)[has] == 1)


def test_alpha_monotone_in_t_max_and_bounded():
    rgba, depth, src, dst = synth.source_image(synth.TINY)
    cr, colour, _ = oracle.unproject(src, rgba, depth, 1.0, half=False)
    prev = None
    for t_max in [1.0, 1.9, 2.1, 2.3, 2.6, np.inf]:
        out = oracle.render(cr, colour, dst, alpha_stop=0.99, t_max=t_max)
        A = out["rgba"][:, 3]
        C = out["rgba"][:, :3]
        assert np.all(C >= 0) and np.all(C <= A[:, None] + 1e-12) and np.all(A <= 1 + 1e-12)
        if prev is not None:
            assert np.all(A >= prev - 1e-12)
        prev = A
    assert prev.max() > 0.5


def test_depth_complexity_bounded_by_seven():
    """Every splat has alpha >= 0.5, so constant-alpha compositing stops within 7 hits."""
    rgba, depth, src, dst = synth.source_image(synth.TINY)
    cr, colour, _ = oracle.unproject(src, rgba, depth, 2.0, half=False)
    assert colour[:, 3].min() >= 0.5
    out = oracle.render(cr, colour, dst, alpha_stop=0.99)
    assert out["n"].max() <= 7
    assert out["n"].max() >= 2
