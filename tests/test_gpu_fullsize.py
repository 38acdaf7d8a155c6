"""Parity at the benchmark's full size (1,000,000 primitives, K = 4, SH degree
3, 1297x840), in the launch configuration bench.py times, on outputs the
oracle can compute one by one: seeded sampled tiles for the forward, seeded
sampled primitives for the backward, the whole frame for the loss."""
import numpy as np
import pytest
import torch

import synth
from oracle import gabor_oracle as O

from gpu_helpers import compare_image, last_ids_from_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    from paper_2508_05343_amd.rasterize import DeviceScene, RenderPlan
    sc, cam = synth.config2_scene(), synth.config2_camera()
    ds = DeviceScene.from_host(sc)
    plan = RenderPlan([ds], [cam])
    plan.forward()
    torch.cuda.synchronize()
    with torch.no_grad():
        pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    return sc, cam, ds, plan, pr


def test_config2_depth_keys_and_visibility(gpu_lib, big):
    sc, cam, ds, plan, pr = big
    d = plan.depth.cpu().numpy()[:sc.n]
    assert (d.view(np.uint32) == pr.depth32.view(np.uint32)).all()
    vis_g = plan.tiles_touched.cpu().numpy()[:sc.n] > 0
    vis_o = pr.visible.numpy()
    assert ((vis_g == vis_o) | pr.fragile_rect).all()
    P = int(plan.num_pairs.item())
    non_fragile = vis_o & ~pr.fragile_rect
    g_tiles = plan.tiles_touched.cpu().numpy()[:sc.n]
    assert (g_tiles[non_fragile] == pr.tiles[non_fragile]).all()
    print(f"visible {vis_o.sum()} pairs {P} fragile rects {pr.fragile_rect.sum()}")


def test_config2_heaviest_tiles_binned_order(gpu_lib, big):
    """The tiles with the most pairs (chosen from the oracle's rects) come out
    of the GPU binning in the oracle's (depth, index) order, item for item
    (items with a fragile rect are left out of both lists)."""
    sc, cam, ds, plan, pr = big
    vis = pr.visible.numpy()
    cnt = np.zeros((cam.tiles_y, cam.tiles_x), np.int64)
    for x0, y0, x1, y1 in pr.rect[vis]:
        cnt[y0:y1, x0:x1] += 1
    heavy = np.argsort(cnt.ravel())[::-1][:6]
    assert cnt.ravel()[heavy[0]] > 512  # the longest segments take the 1024-key register sort
    order = O.depth_order(pr.depth32, vis)
    ranges = plan.ranges.cpu().numpy().view(np.uint32)
    vals = plan.vals.cpu().numpy().view(np.uint32)
    frag = pr.fragile_rect
    for t in heavy:
        tx, ty = int(t % cam.tiles_x), int(t // cam.tiles_x)
        ref = O.tile_candidates(pr, order, tx, ty)
        got = vals[ranges[t, 0]:ranges[t, 1]].astype(np.int64)
        ref, got = ref[~frag[ref]], got[~frag[got]]
        assert np.array_equal(got, ref), (tx, ty, len(got), len(ref))


def test_config2_sampled_tiles_forward(gpu_lib, big):
    sc, cam, ds, plan, pr = big
    rng = np.random.Generator(np.random.PCG64(2024))
    sel = rng.choice(cam.num_tiles, size=48, replace=False)
    tiles = [(int(s % cam.tiles_x), int(s // cam.tiles_x)) for s in sel]
    tiles += [(cam.tiles_x - 1, cam.tiles_y - 1), (cam.tiles_x - 1, 0), (0, cam.tiles_y - 1)]  # ragged edges
    with torch.no_grad():
        ref = O.render(None, O.camera_tensors(cam), "binned", tiles=tiles, scene_f32=sc, pr=pr)
    img = plan.view_image(0).cpu().numpy()
    err, frag, nbad = compare_image(img, ref)
    print(f"config2 sampled: max err {err:.3e} fragile {frag:.4f} bad {nbad}")
    assert nbad == 0 and err <= 1e-4
    valid = ~np.isnan(ref.color.numpy()[0]) & ~ref.fragile
    ids = last_ids_from_gpu(plan, 0)
    assert (ids[valid] == ref.last_id[valid]).all()


def test_config3_sampled_primitive_gradients(gpu_lib, big):
    """render_bwd at full size with a seeded image gradient: the gradients of
    200 seeded visible primitives (every attribute) against the oracle's
    exact windowed fp64 gradients."""
    sc, cam, ds, plan, pr = big
    g_img = synth.random_dl_dimage(1003, (3, cam.height, cam.width))
    names = ("means", "scales", "quats", "opacities", "sh", "freqs", "weights")
    grads = {n: torch.zeros_like(getattr(ds, n)) for n in names}
    plan.backward(torch.from_numpy(g_img.reshape(-1)).cuda(), [grads], accumulate=False)
    torch.cuda.synchronize()
    vis = np.nonzero(pr.visible.numpy() & (pr.tiles <= 9) & ~pr.fragile_prim)[0]
    rng = np.random.Generator(np.random.PCG64(3003))
    prims = rng.choice(vis, size=200, replace=False)
    ref = O.primitive_grads_windowed(sc, cam, g_img, prims, pr_all=pr)
    n = sc.n
    gpu = {}
    gpu["means"] = grads["means"].cpu().numpy()[:, prims].T
    gpu["scales"] = grads["scales"].cpu().numpy()[:, prims].T
    gpu["quats"] = grads["quats"].cpu().numpy()[:, prims].T
    gpu["opacities"] = grads["opacities"].cpu().numpy()[prims]
    gpu["sh"] = grads["sh"].cpu().numpy().reshape(n, 16, 3)[prims]
    gpu["freqs"] = grads["freqs"].cpu().numpy().reshape(4, 3, n)[:, :, prims].transpose(2, 0, 1)
    gpu["weights"] = grads["weights"].cpu().numpy()[:, prims].T
    rep = {}
    for name in names:
        r = np.stack([ref[j][name] for j in range(len(prims))])
        a = gpu[name].reshape(r.shape)
        rep[name] = np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30)
    print({k: f"{v:.2e}" for k, v in rep.items()})
    for name, rel in rep.items():
        assert rel <= 1e-3, (name, rel)


def test_config3_loss_full_frame(gpu_lib, big):
    from paper_2508_05343_amd.rasterize import LossBuffers
    sc, cam, ds, plan, pr = big
    # seeded image and target of the full frame size (no input comes from the GPU path)
    x = synth.random_target(77, (3, cam.height, cam.width))
    tgt = synth.random_target(1003, (3, cam.height, cam.width))
    lb = LossBuffers(3, cam.height, cam.width)
    L, g = lb(torch.from_numpy(x).cuda(), torch.from_numpy(tgt).cuda())
    torch.cuda.synchronize()
    Lr, gr = O.loss_and_grad(x, tgt)
    assert abs(float(L.item()) - Lr) <= 1e-5 * abs(Lr)
    ga = g.cpu().numpy()
    assert np.linalg.norm(ga - gr) / np.linalg.norm(gr) <= 1e-4
