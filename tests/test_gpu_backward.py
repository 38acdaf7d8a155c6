"""GPU backward parity (K7 + K8) and the photometric loss (K9) against the
CPU oracle's exact fp64 derivatives, through the C ABI."""
import numpy as np
import pytest
import torch

import synth
from oracle import gabor_oracle as O

from gpu_helpers import assert_image, check_grads_elementwise, gpu_plan, oracle_project

pytestmark = pytest.mark.gpu

NAMES = ("means", "scales", "quats", "opacities", "sh", "colors", "freqs", "weights")


def _gpu_grads(ds, plan, g_img):
    sc = ds[0]
    grads = {n: torch.zeros_like(getattr(sc, n)) for n in NAMES if getattr(sc, n, None) is not None}
    plan.backward(torch.from_numpy(np.ascontiguousarray(g_img, np.float32).reshape(-1)).cuda(), [grads])
    torch.cuda.synchronize()
    return grads


def _to_aos(name, t, n, k):
    a = t.detach().cpu().numpy()
    if name == "opacities":
        return a
    if name == "sh":  # colour arrays are stored one row per primitive
        return a.reshape(n, -1, 3)
    if name == "colors":
        return a
    if name == "freqs":
        return a.reshape(k, 3, n).transpose(2, 0, 1)
    return a.T


def _check_grads(sc, cam, seed, tol=1e-3, scene_name=""):
    ds, plan = gpu_plan(sc, [cam])
    plan.forward()
    g_img = synth.random_dl_dimage(seed, (3, cam.height, cam.width))
    gg = _gpu_grads(ds, plan, g_img)
    ref = O.render_grads(sc, cam, g_img, "binned")
    slack = O.render_grad_slack(sc, cam, g_img)
    report = {}
    for name, t in gg.items():
        report[name] = check_grads_elementwise(name, _to_aos(name, t, sc.n, sc.k), ref[name], slack[name],
                                               norm_tol=tol)
    print(scene_name, {k: f"out {v[0]} worst {v[1]:.2f} l2 {v[2]:.2e}" for k, v in report.items()})


@pytest.mark.parametrize("deg", [0, 2])
def test_backward_small_sh_scene(gpu_lib, deg):
    """Colour rows of 3 and 27 floats: the one-float-at-a-time row paths."""
    sc = synth.uniform_scene(41, 300, 2, sh_degree=deg, log_scale_mu=-2.6)
    cam = synth.pinhole_camera(64, 48, 60.0, eye=(0.0, 0.0, -3.0), target=(0.0, 0.0, 0.0), bg=(0.1, 0.2, 0.3))
    _check_grads(sc, cam, 5, scene_name=f"sh{deg} k2")


def test_backward_1k_scene(gpu_lib):
    _check_grads(synth.scene_1k_k2_rgb(), synth.camera_128(), 6, scene_name="1k scene")


def test_backward_k4_sh3_rotated_camera(gpu_lib):
    sc = synth.uniform_scene(42, 800, 4, sh_degree=3, log_scale_mu=-3.0)
    cam = synth.pinhole_camera(96, 80, 50.0, eye=(1.2, -0.7, -2.5), target=(0.1, 0.0, 0.2), bg=(1.0, 1.0, 1.0))
    _check_grads(sc, cam, 7, scene_name="sh3 k4")


@pytest.mark.parametrize("k", [0, 1, 5, 8])
def test_forward_and_backward_every_component_count(gpu_lib, k):
    """K = 0 (the Gaussian special case: 10 reduced components), 1, 5 and 8
    (34 components, 11 staged float4s per record): image and gradients
    against the oracle."""
    sc = synth.uniform_scene(60 + k, 400, k, sh_degree=1, log_scale_mu=-2.9)
    cam = synth.pinhole_camera(56, 40, 60.0, eye=(0.3, -0.2, -3.0), target=(0.0, 0.0, 0.0), bg=(0.2, 0.1, 0.3))
    ds, plan = gpu_plan(sc, [cam])
    plan.forward()
    torch.cuda.synchronize()
    ref = O.render_scene(sc, cam, "binned")
    assert_image(plan.view_image(0).cpu().numpy(), ref, f"k{k}")
    _check_grads(sc, cam, 70 + k, scene_name=f"k{k}")


def test_wide_frequency_records(gpu_lib):
    """Records whose image-plane frequencies reach 45 cycles/px (|fx| + |fy|
    above 33, so a tile's phases can leave [-256, 256] cycles) take the
    blend's per-pixel phase reduction; the rest take the unreduced phases.
    Both kinds in one frame: image and gradients against the oracle.  Phases
    of ~340 cycles carry ~2e-5 cycles of float32 rounding (~1.3e-4 in a
    cosine, up to ~3% of the 1/255 alpha threshold), so decisions within 5%
    of a threshold are fragile here and the bounds are scaled to that error."""
    sc = synth.uniform_scene(71, 300, 2, sh_degree=1, log_scale_mu=-2.6)
    cam = synth.pinhole_camera(64, 48, 60.0, eye=(0.0, 0.0, -3.0), target=(0.0, 0.0, 0.0), bg=(0.1, 0.2, 0.3))
    pr = oracle_project(sc, cam)
    m = np.abs(pr.f2d.numpy()).sum(-1).max(1)  # per primitive, max_k |fx| + |fy| (cycles/px)
    sel = np.random.default_rng(0).random(sc.n) < 0.5
    sc.freqs = (sc.freqs * np.where(sel, 45.0 / np.maximum(m, 1e-6), 1.0)[:, None, None]).astype(np.float32)
    pr = oracle_project(sc, cam)
    m = np.abs(pr.f2d.numpy()).sum(-1).max(1)
    vis = pr.visible.numpy()
    wide = 7.5 * m + 0.5 > 250.0
    assert (wide & vis).sum() > 50 and (~wide & vis).sum() > 50
    ds, plan = gpu_plan(sc, [cam])
    plan.forward()
    ref = O.render_scene(sc, cam, "binned", tau_alpha=0.05)
    assert_image(plan.view_image(0).cpu().numpy(), ref, "wide frequencies", atol=1e-3, max_fragile=0.25)
    g_img = synth.random_dl_dimage(72, (3, cam.height, cam.width))
    gg = _gpu_grads(ds, plan, g_img)
    rg = O.render_grads(sc, cam, g_img, "binned")
    report = {}
    for name, t in gg.items():
        report[name] = check_grads_elementwise(name, _to_aos(name, t, sc.n, sc.k), rg[name], rel=1e-2,
                                               max_outlier_frac=0.05, norm_tol=2e-2)
    print("wide", {k: f"out {v[0]} worst {v[1]:.2f} l2 {v[2]:.2e}" for k, v in report.items()})


def test_loss_matches_oracle(gpu_lib):
    from paper_2508_05343_amd.rasterize import LossBuffers
    for (c, h, w, seed) in [(3, 40, 56, 1), (3, 17, 33, 2), (1, 5, 7, 3)]:
        x = synth.random_target(seed, (c, h, w))
        y = synth.random_target(seed + 100, (c, h, w))
        x[0, :3, :3] = y[0, :3, :3]  # equal pixels: zero L1 gradient
        lb = LossBuffers(c, h, w)
        L, g = lb(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
        torch.cuda.synchronize()
        Lr, gr = O.loss_and_grad(x, y)
        assert abs(float(L.item()) - Lr) <= 1e-5 * abs(Lr) + 1e-7
        ga = g.cpu().numpy()
        assert np.linalg.norm(ga - gr) / np.linalg.norm(gr) <= 1e-4
        assert np.abs(ga - gr).max() <= 1e-4 * np.abs(gr).max()


@pytest.mark.parametrize("high_freq", [False, True])
def test_attenuated_forward_and_backward(gpu_lib, high_freq):
    """GABSPLAT_FLAG_ATTENUATION: forward and every gradient against the
    oracle's attenuation-corrected projection."""
    from paper_2508_05343_amd.rasterize import DeviceScene, RenderPlan
    sc = synth.uniform_scene(44, 500, 3, sh_degree=1, log_scale_mu=-2.7)
    if high_freq:
        sc.freqs *= 4.0
    cam = synth.pinhole_camera(64, 56, 55.0, eye=(0.5, -0.3, -2.8), target=(0.0, 0.0, 0.0), bg=(0.3, 0.3, 0.3))
    ds = DeviceScene.from_host(sc, attenuation=True)
    plan = RenderPlan([ds], [cam])
    plan.forward()
    ref = O.render_scene(sc, cam, "binned", attenuation=True)
    assert_image(plan.view_image(0).cpu().numpy(), ref, f"attenuated, high_freq={high_freq}")
    g_img = synth.random_dl_dimage(45, (3, cam.height, cam.width))
    gg = _gpu_grads([ds], plan, g_img)
    rg = O.render_grads(sc, cam, g_img, "binned", attenuation=True)
    sl = O.render_grad_slack(sc, cam, g_img, attenuation=True)
    for name, t in gg.items():
        check_grads_elementwise(name, _to_aos(name, t, sc.n, sc.k), rg[name], sl[name])


def test_unaligned_colour_rows(gpu_lib):
    """SH rows that do not start on a 16-byte boundary (a view one float into
    a buffer) take the float-at-a-time row loads: the same image, bit for bit,
    and the same gradients up to the order of the backward's atomic adds."""
    from paper_2508_05343_amd.rasterize import DeviceScene, RenderPlan
    sc = synth.uniform_scene(45, 400, 2, sh_degree=3, log_scale_mu=-2.8)
    cam = synth.pinhole_camera(64, 48, 60.0, eye=(0.0, 0.0, -3.0), target=(0.0, 0.0, 0.0), bg=(0.1, 0.2, 0.3))
    ds = DeviceScene.from_host(sc)

    def shifted(t):
        buf = torch.zeros(t.numel() + 1, dtype=t.dtype, device=t.device)
        buf[1:].copy_(t.reshape(-1))
        return buf[1:].view(t.shape)
    ds2 = DeviceScene(ds.means, ds.scales, ds.quats, ds.opacities, ds.freqs, ds.weights, sh=shifted(ds.sh),
                      sh_degree=ds.sh_degree)
    assert ds2.sh.data_ptr() % 16 != 0
    g = torch.from_numpy(synth.random_dl_dimage(46, (3 * cam.height * cam.width,))).cuda()
    out = []
    for d in (ds, ds2):
        plan = RenderPlan([d], [cam])
        img = plan.forward().clone()
        grads = {n: torch.zeros_like(getattr(d, n)) for n in NAMES if getattr(d, n, None) is not None}
        grads["sh"] = shifted(grads["sh"])
        plan.backward(g, [grads], accumulate=False)
        torch.cuda.synchronize()
        out.append((img, grads))
    assert torch.equal(out[0][0], out[1][0])
    for n, a in out[0][1].items():
        b = out[1][1][n]
        scale = float(a.abs().max())
        assert float((a - b).abs().max()) <= 1e-5 * scale + 1e-7, n


@pytest.mark.parametrize("lo,hi,seed,log_s,wmax,n", [(0.995, 0.9999, 300, 0.6, 0.01, 150),
                                                    (0.3, 0.6, 301, -0.6, 0.1, 120)])
def test_backward_stacked_opaque_primitives(gpu_lib, lo, hi, seed, log_s, wmax, n):
    """Large primitives stacked in front of the camera.  With opacities in
    [0.995, 0.9999] alpha reaches its 0.99 clamp near the centres and a
    quarter of the pixels stop after two or three blends with T near 1e-4;
    with [0.3, 0.6] the chains run over up to ~120 primitives.  The backward
    recovers every T_i by division from the final transmittance: the image,
    final T and every gradient element against the oracle.  Two clamped
    records leave T (1 - alpha) exactly at the 1e-4 threshold in the oracle's
    arithmetic (just under it in float32), so the first stack has more fragile
    pixels than a natural scene (each is bounded, not dropped)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = 2
    means = np.stack([rng.uniform(-0.25, 0.25, n), rng.uniform(-0.2, 0.2, n), rng.uniform(-0.5, 1.5, n)], 1)
    sc = synth.Scene(means=means.astype(np.float32),
                     scales=np.exp(rng.normal(log_s, 0.2, (n, 3))).astype(np.float32),
                     quats=rng.normal(size=(n, 4)).astype(np.float32),
                     opacities=rng.uniform(lo, hi, n).astype(np.float32),
                     freqs=rng.normal(0.0, 1.0, (n, k, 3)).astype(np.float32),
                     weights=rng.uniform(0.0, wmax, (n, k)).astype(np.float32),
                     sh=rng.normal(0.0, 0.3, (n, 4, 3)).astype(np.float32))
    cam = synth.pinhole_camera(64, 48, 60.0, eye=(0.0, 0.0, -3.0), target=(0.0, 0.0, 0.0), bg=(0.1, 0.2, 0.3))
    ds, plan = gpu_plan(sc, [cam])
    plan.forward()
    torch.cuda.synchronize()
    ref = O.render_scene(sc, cam, "binned")
    assert_image(plan.view_image(0).cpu().numpy(), ref, f"stack [{lo}, {hi}]", max_fragile=0.03)
    ok = ~ref.fragile
    T = plan.view_final_T(0).cpu().numpy()
    Tr = ref.final_T.numpy()
    assert (np.abs(T - Tr)[ok] <= 1e-4 * Tr[ok] + 1e-9).all()
    nb = ref.n_blended
    print("blended per pixel: min", nb.min(), "max", nb.max(), "final T min", float(Tr.min()))
    if lo >= 0.99:
        assert ((nb <= 3) & (Tr < 1e-3)).mean() > 0.2
    else:
        assert nb.max() >= 100
    _check_grads(sc, cam, seed + 1, scene_name=f"stack [{lo}, {hi}]")
