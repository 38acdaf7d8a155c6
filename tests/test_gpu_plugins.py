"""GPU parity of the plug-in variants (Mip-Splatting's 3D and 2D filters, the
3D filter variance, the AbsGS homodirectional gradient and split rule)
against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import synth
from oracle import density_oracle as D
from oracle import gabor_oracle as O

from gpu_helpers import assert_image, check_grads_elementwise, record_fields_np

pytestmark = pytest.mark.gpu

NAMES = ("means", "scales", "quats", "opacities", "sh", "colors", "freqs", "weights")


def _variances(seed, n, lo=1e-5, hi=2e-3):
    """Seeded filter variances (world units squared) of the size the sampling
    rate of a 60-degree 64-pixel camera at depth 3 gives (about 1e-3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n)).astype(np.float32)


def _plan(sc, cams, mip2d=False, filter3d=None, abs_mean2d=False):
    from paper_2508_05343_amd.rasterize import DeviceScene, RenderPlan
    ds = DeviceScene.from_host(sc, mip2d=mip2d)
    if filter3d is not None:
        ds.filter3d = torch.from_numpy(filter3d).cuda()
    return ds, RenderPlan([ds], cams, abs_mean2d=abs_mean2d)


def _cameras():
    return [synth.pinhole_camera(64, 48, 60.0, (0.0, 0.0, -3.0), (0.0, 0.0, 0.0), bg=(0.1, 0.2, 0.3)),
            synth.pinhole_camera(96, 80, 50.0, (1.2, -0.7, -2.5), (0.1, 0.0, 0.2)),
            synth.pinhole_camera(40, 40, 70.0, (-2.0, 0.3, 1.0), (0.0, 0.0, 0.0)),
            synth.pinhole_camera(50, 30, 40.0, (0.0, 2.5, -1.0), (0.0, 0.0, 0.0))]


def test_filter3d_variances_match_oracle(gpu_lib):
    from paper_2508_05343_amd.rasterize import DeviceScene
    sc = synth.uniform_scene(81, 5000, 2, sh_degree=0, log_scale_mu=-3.0)
    sc.means[:50] = sc.means[:50] * 0.1 + np.float32([0.0, 0.0, -40.0])  # behind every camera: unseen
    cams = _cameras()
    ds = DeviceScene.from_host(sc)
    var = ds.compute_filter3d(cams, 0.2, 0.15)
    torch.cuda.synchronize()
    ref, frag = O.mip_filter3d(sc.means, cams, 0.2, 0.15)
    g = var.cpu().numpy()[:sc.n]
    assert not frag[:50].any() and frag.mean() < 0.01
    assert (ref[:50] == ref[50:].max()).all()  # the case holds unseen primitives
    ok = ~frag
    np.testing.assert_allclose(g[ok], ref[ok], rtol=2e-6)
    # a second call on the same tensor (the plans keep its pointer)
    var2 = ds.compute_filter3d(cams[:1], 0.3, 0.0)
    torch.cuda.synchronize()
    assert var2.data_ptr() == var.data_ptr()
    ref2, frag2 = O.mip_filter3d(sc.means, cams[:1], 0.3, 0.0)
    np.testing.assert_allclose(var2.cpu().numpy()[~frag2], ref2[~frag2], rtol=2e-6)


@pytest.mark.parametrize("mip2d,mip3d", [(True, False), (False, True), (True, True)])
def test_filtered_forward_matches_oracle(gpu_lib, mip2d, mip3d):
    sc = synth.uniform_scene(82, 800, 4, sh_degree=3, log_scale_mu=-3.2)
    cam = synth.pinhole_camera(96, 80, 50.0, (1.2, -0.7, -2.5), (0.1, 0.0, 0.2), bg=(0.3, 0.3, 0.3))
    fv = _variances(83, sc.n) if mip3d else None
    ds, plan = _plan(sc, [cam], mip2d, fv)
    plan.forward()
    torch.cuda.synchronize()
    with torch.no_grad():
        pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc, mip2d=mip2d, filter3d=fv)
    tiles = plan.tiles_touched.cpu().numpy()[:sc.n]
    vis_o, frag = pr.visible.numpy(), pr.fragile_rect
    assert (((tiles > 0) == vis_o) | frag).all()
    rect = plan.rect.cpu().numpy()[:sc.n].astype(np.int64)
    rg = np.stack([rect[:, 0] & 0xFFFF, rect[:, 0] >> 16, rect[:, 1] & 0xFFFF, rect[:, 1] >> 16], 1)
    sel = vis_o & (tiles > 0) & ~frag
    assert (rg[sel] == pr.rect[sel]).all()
    f = record_fields_np(plan)
    m = sel & ~pr.fragile_prim
    assert m.sum() > 100
    np.testing.assert_allclose(f["opacity"][m], pr.opac.numpy()[m], rtol=2e-5)
    con = pr.conic.numpy()[m]
    assert (np.abs(f["conic"][m] - con) <= 2e-5 * np.abs(con).max(1, keepdims=True) + 1e-9).all()
    f2 = pr.f2d.numpy()[m]
    assert (np.abs(f["f2d"][m] - f2) <= 2e-5 * (np.abs(f2).max(axis=(1, 2), keepdims=True) + 1e-6)).all()
    ref = O.render_scene(sc, cam, "binned", mip2d=mip2d, filter3d=fv)
    assert_image(plan.view_image(0).cpu().numpy(), ref, f"mip2d {mip2d} mip3d {mip3d}")


@pytest.mark.parametrize("mip2d,mip3d", [(True, False), (False, True), (True, True)])
def test_filtered_backward_matches_oracle(gpu_lib, mip2d, mip3d):
    sc = synth.uniform_scene(84, 600, 2, sh_degree=2, log_scale_mu=-3.0)
    cam = synth.pinhole_camera(64, 48, 60.0, (0.0, 0.0, -3.0), (0.0, 0.0, 0.0), bg=(0.1, 0.2, 0.3))
    fv = _variances(85, sc.n) if mip3d else None
    ds, plan = _plan(sc, [cam], mip2d, fv)
    plan.forward()
    g_img = synth.random_dl_dimage(86, (3, cam.height, cam.width))
    grads = {n: torch.zeros_like(getattr(ds, n)) for n in NAMES if getattr(ds, n, None) is not None}
    plan.backward(torch.from_numpy(np.ascontiguousarray(g_img, np.float32).reshape(-1)).cuda(), [grads])
    torch.cuda.synchronize()
    ref = O.render_grads(sc, cam, g_img, "binned", mip2d=mip2d, filter3d=fv)
    slack = O.render_grad_slack(sc, cam, g_img, mip2d=mip2d, filter3d=fv)
    for name, t in grads.items():
        a = t.detach().cpu().numpy()
        if name == "sh":  # one row per primitive
            a = a.reshape(sc.n, -1, 3)
        elif name == "freqs":
            a = a.reshape(-1, 3, sc.n).transpose(2, 0, 1)
        elif name not in ("opacities", "colors"):
            a = a.T
        check_grads_elementwise(name, a, ref[name], slack[name])


def test_abs_mean_gradient_matches_oracle(gpu_lib):
    """grad2d of an abs_mean2d plan: the mean columns equal the oracle's summed
    per-pixel gradients, the two extra columns its sums of absolute values; the
    scene gradients equal those of a plain plan."""
    for (k, seed) in ((0, 86), (2, 87), (4, 88), (8, 89)):
        sc = synth.uniform_scene(seed, 500, k, sh_degree=1, log_scale_mu=-3.0)
        cam = synth.pinhole_camera(64, 48, 60.0, (0.0, 0.0, -3.0), (0.0, 0.0, 0.0), bg=(0.1, 0.2, 0.3))
        g_img = synth.random_dl_dimage(seed + 1, (3, cam.height, cam.width))
        dl = torch.from_numpy(np.ascontiguousarray(g_img, np.float32).reshape(-1)).cuda()
        outs = []
        for abs_on in (False, True):
            ds, plan = _plan(sc, [cam], abs_mean2d=abs_on)
            plan.forward()
            grads = {n: torch.zeros_like(getattr(ds, n)) for n in NAMES if getattr(ds, n, None) is not None}
            plan.backward(dl, [grads])
            torch.cuda.synchronize()
            outs.append((plan, grads))
        plan = outs[1][0]
        from paper_2508_05343_amd import _lib
        assert plan.grad2d.shape[1] == _lib.gabsplat_grad2d_stride(k, _lib.GRAD_ABS_MEAN2D)
        for name in outs[0][1]:
            a, b = outs[1][1][name].cpu().numpy(), outs[0][1][name].cpu().numpy()
            assert np.linalg.norm(a - b) <= 1e-5 * max(np.linalg.norm(b), 1e-30), name
        tot, ab = O.mean2d_grads(sc, cam, g_img)
        sl = O.render_grad_slack(sc, cam, g_img, with_mean2d=True)["mean2d"]
        vis = plan.tiles_touched.cpu().numpy()[:sc.n] > 0
        g2 = plan.grad2d.cpu().numpy()[:sc.n]
        c = 10 + 3 * k
        for nm, got, want in (("mean2d", g2[vis, 0:2], tot[vis]), ("abs mean2d", g2[vis, c:c + 2], ab[vis])):
            print("k", k, nm, check_grads_elementwise(nm, got, want, sl[vis]))
        assert (g2[vis, c:c + 2] >= np.abs(g2[vis, 0:2]) * (1 - 1e-4) - 1e-9).all()


def test_abs_statistic_and_split_rule_match_oracle(gpu_lib):
    from paper_2508_05343_amd import _lib
    from paper_2508_05343_amd.density import DensityStats, default_params, densify
    from paper_2508_05343_amd.rasterize import DeviceScene, RenderPlan
    sc = synth.uniform_scene(90, 3000, 2, sh_degree=1, log_scale_mu=-4.6, log_scale_sigma=1.0)
    cams = [synth.pinhole_camera(64, 48, 60.0, (0, 0, -3.0), (0, 0, 0)),
            synth.pinhole_camera(40, 40, 60.0, (1.0, 0, -3.0), (0, 0, 0))]
    ds = DeviceScene.from_host(sc)
    plan = RenderPlan([ds], cams, [0, 0], abs_mean2d=True)
    plan.preprocess()
    rng = np.random.Generator(np.random.PCG64(91))
    gf = _lib.gabsplat_grad2d_stride(sc.k, _lib.GRAD_ABS_MEAN2D)
    g2 = rng.normal(0, 1e-3, size=(plan.items, gf)).astype(np.float32)
    c = 10 + 3 * sc.k
    g2[:, c:c + 2] = np.abs(g2[:, 0:2]) * rng.uniform(1.0, 3.0, (plan.items, 2)).astype(np.float32)
    tiles = (rng.uniform(size=plan.items) < 0.6).astype(np.int32) * rng.integers(1, 5, plan.items).astype(np.int32)
    plan.grad2d = torch.from_numpy(g2).cuda()
    plan.tiles_touched.copy_(torch.from_numpy(tiles).cuda())
    st = DensityStats(sc.n, abs_stat=True)
    st.accumulate(plan)
    torch.cuda.synchronize()
    acc, den, acc_abs = np.zeros(sc.n), np.zeros(sc.n), np.zeros(sc.n)
    for v, cm in enumerate(cams):
        sl = slice(v * sc.n, (v + 1) * sc.n)
        D.accumulate_stats(g2[sl, 0:2], tiles[sl] > 0, cm.width, cm.height, acc, den, g2[sl, c:c + 2], acc_abs)
    np.testing.assert_allclose(st.accum.cpu().numpy(), acc, rtol=1e-5, atol=1e-12)
    np.testing.assert_allclose(st.accum_abs.cpu().numpy(), acc_abs, rtol=1e-5, atol=1e-12)
    np.testing.assert_array_equal(st.denom.cpu().numpy(), den)
    # the split rule on seeded statistics
    rng = np.random.Generator(np.random.PCG64(92))
    denom = rng.integers(0, 4, sc.n).astype(np.float32)
    accum = (rng.exponential(0.0002, sc.n) * denom).astype(np.float32)
    accum_abs = (accum * rng.uniform(1.0, 4.0, sc.n)).astype(np.float32)
    normals = rng.normal(size=(sc.n, 2, 3)).astype(np.float32)
    st2 = DensityStats(sc.n, abs_stat=True)
    st2.accum.copy_(torch.from_numpy(accum))
    st2.denom.copy_(torch.from_numpy(denom))
    st2.accum_abs.copy_(torch.from_numpy(accum_abs))
    nrm = torch.from_numpy(np.ascontiguousarray(normals.transpose(1, 2, 0).reshape(-1))).cuda()
    new, src, tag = densify(ds, st2, nrm, default_params(abs_grad_threshold=0.0004))
    torch.cuda.synchronize()
    prm = D.DensifyParams(abs_grad_threshold=0.0004)
    ref, rsrc, rtag = D.densify(sc, accum, denom, normals, prm, accum_abs)
    kinds = D.decide(sc, accum, denom, prm, accum_abs)
    plain = D.decide(sc, accum, denom, D.DensifyParams())
    assert ((kinds == 2) & (plain == 0)).any()  # the case exercises the absolute statistic
    assert new.n == len(rsrc)
    np.testing.assert_array_equal(src.cpu().numpy(), rsrc)
    np.testing.assert_array_equal(tag.cpu().numpy(), rtag)
    means = new.means.cpu().numpy().T
    orig = rtag <= 1
    np.testing.assert_array_equal(means[orig], ref["means"][orig].astype(np.float32))
    np.testing.assert_allclose(means[~orig], ref["means"][~orig], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(new.scales.cpu().numpy().T, ref["scales"], rtol=1e-6)
