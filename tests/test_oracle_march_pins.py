"""Pins of the oracle's server ray marcher (the stage before the path, Sec.
3.1) against closed forms and an independent implementation:
* a constant volume composites as 1 - (1 - s)^k, with the depth at a known
  sample;
* trilinear reconstruction reproduces a linear ramp and clamps at the edges;
* a ray that misses the cube, or starts inside it, is handled exactly;
* the input generator's own caster (written separately) gives the same
  image."""
import math

import numpy as np
import pytest

import oracle
import synth


def _axis_camera(w, h, eye, forward, up=(0.0, 1.0, 0.0), fov_deg=30.0):
    f = np.array(forward, dtype=np.float64)
    f /= np.linalg.norm(f)
    u = np.array(up, dtype=np.float64)
    r = np.cross(f, u)
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    return synth.Camera(tuple(eye), tuple(f), tuple(r), tuple(u), math.tan(math.radians(fov_deg) / 2), w, h)


def _constant_closed_form(value, t_in, t_out, n, size, alpha_scale=0.05, depth_alpha=0.5, stop_alpha=0.999):
    """(C, A, depth, samples) of the march through a constant volume, from the closed form."""
    s = min(max(alpha_scale * value, 0.0), 1.0)
    u = min(max(value, 0.0), 1.0)
    dt = 0.5 * size / n
    k_in = max(0, math.ceil((t_out - t_in) / dt - 0.5))  # samples with t_in + (j + 1/2) dt < t_out
    # samples until A = 1 - (1 - s)^k reaches the stop
    k_stop = math.ceil(math.log(1.0 - stop_alpha) / math.log(1.0 - s)) if s > 0 else k_in + 1
    k = min(k_in, k_stop)
    A = 1.0 - (1.0 - s) ** k
    k_depth = math.ceil(math.log(1.0 - depth_alpha) / math.log(1.0 - s)) if s > 0 else k + 1
    depth = t_in + (k_depth - 0.5) * dt if k_depth <= k else math.inf
    colour = np.array([u, 4.0 * u * (1.0 - u), 1.0 - u])
    return colour * A, A, depth, k


@pytest.mark.parametrize("value", [0.6, 1.7, 12.0])
def test_constant_volume_closed_form(value):
    n, lo, size = 32, -0.25, 1.5
    vol = np.full((n, n, n), value, dtype=np.float32)
    # 5x5 view straight down -z through the cube centre: the centre pixel's
    # ray is the axis, entering at z = lo + size and leaving at z = lo
    centre = lo + size / 2
    cam = _axis_camera(5, 5, (centre, centre, 3.0), (0.0, 0.0, -1.0))
    got = oracle.raymarch(vol, lo, size, cam, pixels=[12])
    v32 = float(np.float32(value))  # the value the volume stores
    C, A, depth, _ = _constant_closed_form(v32, 3.0 - (lo + size), 3.0 - lo, n, size)
    assert np.allclose(got["rgba"][0, :3], C, rtol=1e-12, atol=1e-14)
    assert got["rgba"][0, 3] == pytest.approx(A, rel=1e-12)
    if math.isfinite(depth):
        assert got["depth"][0] == pytest.approx(depth, rel=1e-12)
    else:
        assert got["depth"][0] == math.inf


def test_eye_inside_the_volume():
    """Marching starts at t = 0 when the eye is inside the cube."""
    n, lo, size = 32, -0.25, 1.5
    vol = np.full((n, n, n), 0.9, dtype=np.float32)
    centre = lo + size / 2
    cam = _axis_camera(5, 5, (centre, centre, centre), (0.0, 0.0, -1.0))
    got = oracle.raymarch(vol, lo, size, cam, pixels=[12])
    C, A, depth, _ = _constant_closed_form(float(np.float32(0.9)), 0.0, centre - lo, n, size)
    assert got["rgba"][0, 3] == pytest.approx(A, rel=1e-12)
    assert got["depth"][0] == pytest.approx(depth, rel=1e-12)


def test_linear_ramp_is_reproduced_and_clamped():
    n = 16
    x = (np.arange(n) + 0.5) / n  # value = x coordinate of the voxel centre
    vol = np.broadcast_to(x[None, None, :], (n, n, n)).astype(np.float32).copy()
    rng = np.random.default_rng(2)
    for _ in range(50):
        p = rng.uniform(0.5 / n, 1 - 0.5 / n, 3)
        assert oracle.volume_sample(vol, p) == pytest.approx(p[0], abs=1e-12)
    # outside the voxel centres the edge value holds
    assert oracle.volume_sample(vol, [0.0, 0.5, 0.5]) == pytest.approx(float(vol[0, 0, 0]), abs=0)
    assert oracle.volume_sample(vol, [1.0, 0.5, 0.5]) == pytest.approx(float(vol[0, 0, n - 1]), abs=0)


def test_trilinear_weights_on_a_single_voxel_pulse():
    """A single non-zero voxel: the sample equals the product of the three
    hat functions around its centre."""
    n = 8
    vol = np.zeros((n, n, n), dtype=np.float32)
    vol[3, 4, 2] = 1.0  # z, y, x
    rng = np.random.default_rng(5)
    for _ in range(40):
        p = rng.uniform(0.2, 0.8, 3)
        g = p * n - 0.5
        hat = np.maximum(0.0, 1.0 - np.abs(g - np.array([2, 4, 3])))
        assert oracle.volume_sample(vol, p) == pytest.approx(float(np.prod(hat)), abs=1e-12)


def test_ray_missing_the_cube_is_background():
    n, lo, size = 8, -0.25, 1.5
    vol = np.ones((n, n, n), dtype=np.float32)
    cam = _axis_camera(4, 3, (5.0, 5.0, 5.0), (1.0, 1.0, 1.0))  # looking away
    got = oracle.raymarch(vol, lo, size, cam)
    assert np.all(got["rgba"] == 0.0) and np.all(np.isinf(got["depth"]))


def test_stop_never_lowers_alpha_monotone():
    """Without the stop, alpha and colour only grow; the stop cuts after A >= 0.999."""
    vol = synth.volume_of(synth.TINY)
    _, _, src, _ = synth.source_image(synth.TINY)
    a = oracle.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src)
    b = oracle.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src, stop_alpha=2.0)
    assert np.all(b["rgba"][:, 3] >= a["rgba"][:, 3] - 1e-15)
    assert np.all(b["rgba"] >= a["rgba"] - 1e-15)
    assert np.all(a["rgba"][:, 3] <= 1.0)


def test_matches_the_input_generators_caster():
    """The input generator ray-casts the source images with the same rules,
    in code written separately; its float output agrees to float rounding."""
    vol = synth.volume_of(synth.TINY)
    rgba, depth, src, _ = synth.source_image(synth.TINY)
    got = oracle.raymarch(vol, synth.BOX_LO, synth.BOX_SIZE, src)
    assert np.abs(got["rgba"] - rgba.reshape(-1, 4)).max() < 1e-6
    d_ref = depth.reshape(-1).astype(np.float64)
    assert np.array_equal(np.isfinite(got["depth"]), np.isfinite(d_ref))
    fin = np.isfinite(d_ref)
    assert fin.sum() > 100
    assert np.abs(got["depth"][fin] - d_ref[fin]).max() < 1e-6 * np.abs(d_ref[fin]).max()
