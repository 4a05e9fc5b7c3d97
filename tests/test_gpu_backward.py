"""GPU backward (splat_trace_backward): against the oracle's analytic FP64
gradient, against FP64 central differences of the oracle's forward, through
the autograd Function, and a radius/alpha fit to a reference view."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

NEVER = 2.0


@pytest.fixture(scope="module")
def sp():
    import paper_2006_14726_amd as sp
    sp.load_library()
    return sp


def up(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def gpu_grads(sp, cr, col, cam, g, mode, stop):
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    opts = sp.TraceOptions(alpha_stop=stop, mode=mode)
    out, _ = sp.trace(bvh, sph, cam, opts)
    gr = sp.trace_backward(bvh, sph, cam, opts, out, up(g.reshape(cam.height, cam.width, 4).astype(np.float32)))
    torch.cuda.synchronize()
    # oracle order: cx cy cz r kr kg kb a
    return np.concatenate([gr["centre"].cpu().numpy(), gr["radius"].cpu().numpy()[:, None],
                           gr["rgb"].cpu().numpy(), gr["alpha"].cpu().numpy()[:, None]], axis=1).astype(np.float64)


def check_close(gpu, ref, rel=1e-3, floor_frac=1e-2, cols=range(8)):
    """|g - ref| <= rel * max(|ref|, tau), tau = floor_frac * median |ref| of the parameter type."""
    for c in cols:
        r = ref[:, c]
        nz = np.abs(r[r != 0])
        tau = floor_frac * (np.median(nz) if nz.size else 1.0)
        bound = rel * np.maximum(np.abs(r), tau)
        worst = float(np.max(np.abs(gpu[:, c] - r) / bound)) * rel if r.size else 0.0
        print(f"  param {c}: max |g - ref| / max(|ref|, tau) = {worst:.2e}", flush=True)
        bad = np.nonzero(np.abs(gpu[:, c] - r) > bound)[0]
        assert bad.size == 0, f"param {c}: {bad.size} spheres off, e.g. {bad[:5]} gpu {gpu[bad[:5], c]} ref {r[bad[:5]]}"


@pytest.mark.parametrize("mode,stop", [(1, 0.99), (1, NEVER), (0, 0.99), (0, NEVER)])
def test_backward_matches_oracle_gradient(sp, mode, stop):
    cr, col = synth.random_spheres(150, seed=21, r_lo=0.03, r_hi=0.12, a_lo=0.3, a_hi=0.9)
    cam = synth.rotated_camera(synth.source_camera(48, 40), 7.0, 2.0)
    rng = np.random.default_rng(5)
    g = rng.normal(size=(cam.width * cam.height, 4))
    ref = oracle.grad_table(oracle.sphere_table(cr, col), cam, g, alpha_stop=stop, mode=mode)
    gpu = gpu_grads(sp, cr, col, cam, g, mode, stop)
    check_close(gpu, ref, cols=range(8) if mode == 1 else range(4, 8))
    if mode == 0:
        assert np.all(gpu[:, :4] == 0)
    assert np.abs(ref).sum() > 0


def test_backward_with_restarts(sp):
    """Deep overlap: many passes per pixel (k = 1, 2) must give the gradient of one pass."""
    cr, col = synth.random_spheres(300, seed=3, r_lo=0.05, r_hi=0.15, a_lo=0.05, a_hi=0.3)
    cam = synth.rotated_camera(synth.source_camera(32, 24), 5.0)
    g = np.random.default_rng(1).normal(size=(cam.width * cam.height, 4))
    ref = oracle.grad_table(oracle.sphere_table(cr, col), cam, g, alpha_stop=0.99, mode=1)
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    for k, walk in ((1, 0), (2, 1), (6, 0), (16, 1), (4, 2), (16, 2)):
        opts = sp.TraceOptions(mode=1, kbuf=k, walk=walk)
        out, hits = sp.trace(bvh, sph, cam, opts)
        assert int(hits.max()) > 8  # several passes at k = 1 and 2
        gr = sp.trace_backward(bvh, sph, cam, opts, out, up(g.reshape(cam.height, cam.width, 4).astype(np.float32)))
        gpu = np.concatenate([gr["centre"].cpu().numpy(), gr["radius"].cpu().numpy()[:, None],
                              gr["rgb"].cpu().numpy(), gr["alpha"].cpu().numpy()[:, None]], axis=1)
        check_close(gpu.astype(np.float64), ref)


def test_backward_matches_central_differences_on_differentiable_config(sp):
    """512^2 source from the tiny blob generator, reference ray-cast at the target camera,
    L = sum (I - I_ref)^2; 64 probe spheres x 8 parameters against FP64 central differences."""
    work = synth.DIFF
    rgba, depth, src, dst = synth.source_image(work)
    ref_img, _ = synth.raycast(synth.volume_of(work), dst)
    cr, col, _ = oracle.unproject(src, rgba, depth, 1.0, False)
    table = oracle.sphere_table(cr, col)
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    opts = sp.TraceOptions(mode=sp.SPLAT_ALPHA_SOFT)
    out, hits = sp.trace(bvh, sph, dst, opts)
    gout = 2.0 * (out - up(ref_img))
    gr = sp.trace_backward(bvh, sph, dst, opts, out, gout.contiguous())
    torch.cuda.synchronize()
    gpu = np.concatenate([gr["centre"].cpu().numpy(), gr["radius"].cpu().numpy()[:, None],
                          gr["rgb"].cpu().numpy(), gr["alpha"].cpu().numpy()[:, None]], axis=1).astype(np.float64)
    # probes: spheres that take part in at least one pixel
    touched = np.nonzero(np.abs(gpu[:, 7]) > 0)[0]
    rng = np.random.default_rng(4)
    probes = rng.choice(touched, size=min(96, touched.size), replace=False)
    ref_flat = ref_img.reshape(-1, 4).astype(np.float64)
    fd = np.full((probes.size, 8), np.nan)
    skipped = 0
    for i, j in enumerate(probes):
        r = table[j, 3]
        pix = oracle.pixels_near(dst, table[j, :3], r * 1.01)
        for f in range(8):
            h = 1e-4 * (r if f < 4 else 1.0)
            tp, tm = table.copy(), table.copy()
            tp[j, f] += h
            tm[j, f] -= h
            op = oracle.render_table(tp, dst, mode=1, pixels=pix)
            om = oracle.render_table(tm, dst, mode=1, pixels=pix)
            if not (np.array_equal(op["sig"], om["sig"]) and np.array_equal(op["n"], om["n"])):
                skipped += 1
                continue
            lp = ((op["rgba"] - ref_flat[pix]) ** 2).sum()
            lm = ((om["rgba"] - ref_flat[pix]) ** 2).sum()
            fd[i, f] = (lp - lm) / (2 * h)
    ok = ~np.isnan(fd)
    assert ok.sum() >= 64 * 8 * 0.9, f"too many skipped probes: {skipped}"
    g = gpu[probes]
    for f in range(8):
        col_ok = ok[:, f]
        ref = fd[col_ok, f]
        tau = 1e-2 * np.median(np.abs(ref[ref != 0])) if np.any(ref != 0) else 1.0
        err = np.abs(g[col_ok, f] - ref)
        assert np.all(err <= 1e-3 * np.maximum(np.abs(ref), tau)), (f, np.max(err / np.maximum(np.abs(ref), tau)))


def test_autograd_function_matches_direct_backward(sp):
    from paper_2006_14726_amd.autograd import splat_trace
    cr, col = synth.random_spheres(120, seed=8, r_lo=0.04, r_hi=0.12)
    cam = synth.rotated_camera(synth.source_camera(40, 30), 5.0)
    crt, colt = up(cr).requires_grad_(True), up(col).requires_grad_(True)
    sph = sp.spheres_from_tensors(up(cr), up(col))
    bvh = sp.build_bvh(sph)
    opts = sp.TraceOptions(mode=sp.SPLAT_ALPHA_SOFT)
    img = splat_trace(crt, colt, bvh, cam, opts)
    w = torch.randn_like(img)
    (img * w).sum().backward()
    out, _ = sp.trace(bvh, sph, cam, opts)
    gr = sp.trace_backward(bvh, sph, cam, opts, out, w)
    torch.cuda.synchronize()
    assert torch.allclose(crt.grad[:, 3], gr["radius"], rtol=1e-5, atol=1e-6)
    assert torch.allclose(colt.grad[:, 3], gr["alpha"], rtol=1e-5, atol=1e-6)
    assert torch.allclose(colt.grad[:, :3], gr["rgb"], rtol=1e-5, atol=1e-6)
    assert torch.allclose(crt.grad[:, :3], gr["centre"], rtol=1e-5, atol=1e-6)


def test_radius_alpha_fit_reduces_loss(sp):
    """200 Adam steps on (log r, logit a) against the directly ray-cast reference view."""
    from paper_2006_14726_amd.fit import fit_radius_alpha
    work = synth.DIFF
    rgba, depth, src, dst = synth.source_image(work)
    ref_img, _ = synth.raycast(synth.volume_of(work), dst)
    s = sp.unproject(src, up(rgba), up(depth), 1.0, False)
    bvh = sp.build_bvh(s)
    losses = fit_radius_alpha(s, bvh, dst, up(ref_img), steps=200, lr=1e-2)
    print(f"fit loss {losses[0]:.4f} -> {losses[-1]:.4f} ({losses[-1] / losses[0]:.3f})", flush=True)
    assert losses[-1] < 0.9 * losses[0]
