"""Pins of the oracle's analytic gradient: closed forms and FP64 central differences.  CPU only.

The differentiable reading: alpha = a (1 - q/r^2)^2 on the soft profile, the
paper's constant alpha otherwise; the loss is a per-pixel function of the
composited RGBA.
"""
import numpy as np
import pytest

import oracle
import synth
from test_oracle_pins import AXIS_CAM, NEVER, table


def lin_grad(tab, cam, g, mode, alpha_stop=NEVER):
    return oracle.grad_table(tab, cam, np.asarray(g, dtype=np.float64).reshape(-1, 4), alpha_stop=alpha_stop,
                             mode=mode)


def test_soft_alpha_closed_form():
    """c = (0.6, 0, 5), r = 1, a = 0.5: u = 0.36, alpha = 0.5 * 0.64^2 = 0.2048."""
    tab = table([(0.6, 0, 5, 1, 0.25, 0.5, 0.75, 0.5)])
    out = oracle.render_table(tab, AXIS_CAM, alpha_stop=NEVER, mode=oracle.MODE_SOFT)
    assert out["rgba"][0][3] == pytest.approx(0.2048, abs=1e-15)
    assert np.allclose(out["rgba"][0][:3], 0.2048 * np.array([0.25, 0.5, 0.75]), atol=1e-15)
    g = lin_grad(tab, AXIS_CAM, [0, 0, 0, 1], oracle.MODE_SOFT)[0]  # L = A = alpha
    assert g[7] == pytest.approx(0.64 ** 2, abs=1e-14)         # d alpha / d a = (1-u)^2
    assert g[3] == pytest.approx(0.4608, abs=1e-14)            # 4 a (1-u) q / r^3
    assert g[0] == pytest.approx(-0.768, abs=1e-14)            # -4 a (1-u) v_x / r^2
    assert g[1] == pytest.approx(0.0, abs=1e-15) and g[2] == pytest.approx(0.0, abs=1e-15)
    g = lin_grad(tab, AXIS_CAM, [1, 0, 0, 0], oracle.MODE_SOFT)[0]  # L = C_r = alpha k_r
    assert g[4] == pytest.approx(0.2048, abs=1e-15)


def test_two_sphere_constant_alpha_derivatives():
    """C = a1 k1 + (1-a1) a2 k2, A = a1 + (1-a1) a2."""
    a1, a2 = 0.3, 0.6
    k1, k2 = np.array([0.9, 0.2, 0.1]), np.array([0.1, 0.7, 0.4])
    tab = table([(0, 0, 5, 1, *k1, a1), (0, 0, 5.5, 1, *k2, a2)])
    for ch in range(3):
        g = np.zeros(4)
        g[ch] = 1
        gr = lin_grad(tab, AXIS_CAM, g, oracle.MODE_CONSTANT)
        assert gr[0, 7] == pytest.approx(k1[ch] - a2 * k2[ch], abs=1e-15)
        assert gr[1, 7] == pytest.approx((1 - a1) * k2[ch], abs=1e-15)
        assert gr[0, 4 + ch] == pytest.approx(a1, abs=1e-15)
        assert gr[1, 4 + ch] == pytest.approx((1 - a1) * a2, abs=1e-15)
        assert np.all(gr[:, :4] == 0)
    gr = lin_grad(tab, AXIS_CAM, [0, 0, 0, 1], oracle.MODE_CONSTANT)
    assert gr[0, 7] == pytest.approx(1 - a2, abs=1e-15)
    assert gr[1, 7] == pytest.approx(1 - a1, abs=1e-15)


def _loss(tab, cam, g, pix, mode, alpha_stop):
    out = oracle.render_table(tab, cam, alpha_stop=alpha_stop, mode=mode, pixels=pix)
    return float(np.sum(out["rgba"] * g[pix])), out


@pytest.mark.parametrize("mode,alpha_stop", [(oracle.MODE_SOFT, 0.99), (oracle.MODE_SOFT, NEVER),
                                             (oracle.MODE_CONSTANT, 0.99)])
def test_analytic_gradient_matches_central_differences(mode, alpha_stop):
    cr, col = synth.random_spheres(40, seed=9, r_lo=0.06, r_hi=0.18, a_lo=0.3, a_hi=0.9)
    cam = synth.rotated_camera(synth.source_camera(24, 20), 6.0, 2.0)
    tab = oracle.sphere_table(cr, col)
    rng = np.random.default_rng(2)
    g = rng.normal(size=(cam.width * cam.height, 4))
    ana = oracle.grad_table(tab, cam, g, alpha_stop=alpha_stop, mode=mode)
    params = [3, 7, 4, 0, 1, 2] if mode == oracle.MODE_SOFT else [7, 4, 5, 6]
    checked = skipped = 0
    for j in range(tab.shape[0]):
        pix = oracle.pixels_near(cam, tab[j, :3], tab[j, 3] * 1.01)
        if pix.size == 0:
            continue
        for f in params:
            h = 1e-6 * (tab[j, 3] if f < 4 else 1.0)
            tp, tm = tab.copy(), tab.copy()
            tp[j, f] += h
            tm[j, f] -= h
            lp, op = _loss(tp, cam, g, pix, mode, alpha_stop)
            lm, om = _loss(tm, cam, g, pix, mode, alpha_stop)
            if not (np.array_equal(op["sig"], om["sig"]) and np.array_equal(op["n"], om["n"])):
                skipped += 1       # the ordered hit list changes inside the step: L is discontinuous there
                continue
            fd = (lp - lm) / (2 * h)
            assert ana[j, f] == pytest.approx(fd, rel=1e-6, abs=1e-7 * max(1.0, abs(fd))), (j, f)
            checked += 1
    assert checked > 50
    assert skipped <= checked // 10
