"""Parity at the full size of the 64-view training workload (64 views of
800x800, 300,000 primitives, K = 4, SH degree 3): 160,000 tiles in one
launch, so the binning takes the radix path (compaction, depth passes,
tiles-touched scan, emission, tile passes) over ~288M pairs.  Checked on
outputs the oracle can compute one by one: for seeded sampled views, the
binned lists of seeded sampled tiles item for item, and the blended pixels
and last contributors of the same tiles."""
import numpy as np
import pytest
import torch

import synth
from oracle import gabor_oracle as O

from gpu_helpers import assert_dispatch_order, assert_image, check_sampled_grads
from sampling import stratified_primitives

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mv():
    from paper_2508_05343_amd.rasterize import DeviceScene, RenderPlan
    sc, cams = synth.scene_300k_k4_sh3(), synth.orbit_cameras_64x800()
    ds = DeviceScene.from_host(sc)
    plan = RenderPlan([ds], cams)
    plan.forward(check_overflow=True)
    torch.cuda.synchronize()
    return sc, cams, plan


def _tile_lists(plan, v, cam, tiles):
    """The GPU's sorted list of every given tile of view v, as primitive ids."""
    r = plan.view_ranges(v).cpu().numpy().view(np.uint32)
    off = plan.layout[v].item_offset
    out = []
    for tx, ty in tiles:
        t = ty * cam.tiles_x + tx
        a, b = int(r[t, 0]), int(r[t, 1])
        out.append(plan.vals[a:b].cpu().numpy().view(np.uint32).astype(np.int64) - off)
    return out


def test_64_views_sampled_views_binning_and_blend(gpu_lib, mv):
    sc, cams, plan = mv
    assert sum(c.num_tiles for c in cams) > 8192  # the radix path
    assert_dispatch_order(plan)
    rng = np.random.Generator(np.random.PCG64(4004))
    for v in rng.choice(len(cams), size=3, replace=False):
        v = int(v)
        cam = cams[v]
        with torch.no_grad():
            pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
        vis = pr.visible.numpy()
        order = O.depth_order(pr.depth32, vis)
        frag = pr.fragile_rect
        sel = rng.choice(cam.num_tiles, size=8, replace=False)
        tiles = [(int(s % cam.tiles_x), int(s // cam.tiles_x)) for s in sel]
        tiles.append((cam.tiles_x - 1, cam.tiles_y - 1))
        lists = _tile_lists(plan, v, cam, tiles)
        for (tx, ty), got in zip(tiles, lists):
            ref = O.tile_candidates(pr, order, tx, ty)
            assert np.array_equal(got[~frag[got]], ref[~frag[ref]]), (v, tx, ty, len(got), len(ref))
        with torch.no_grad():
            ref = O.render(None, O.camera_tensors(cam), "binned", tiles=tiles, scene_f32=sc, pr=pr)
        img = plan.view_image(v).cpu().numpy()
        # the dense ball saturates most pixels, so more of them take a stop
        # decision near its threshold than in the clustered frame (about 1% of
        # the sampled pixels); every fragile pixel is still held to its bound
        assert_image(img, ref, f"view {v}", max_fragile=0.03)
        # last contributor of every pixel of the sampled tiles
        nc = plan.view_n_contrib(v).cpu().numpy().astype(np.int64)
        valid = ~np.isnan(ref.color.numpy()[0]) & ~ref.fragile
        for (tx, ty), got in zip(tiles, lists):
            ys, xs = slice(ty * 16, min(ty * 16 + 16, cam.height)), slice(tx * 16, min(tx * 16 + 16, cam.width))
            n = nc[ys, xs]
            ids = np.where(n > 0, got[np.clip(n - 1, 0, max(len(got) - 1, 0))] if len(got) else -1, -1)
            ok = valid[ys, xs]
            assert (ids[ok] == ref.last_id[ys, xs][ok]).all(), (v, tx, ty)


def test_64_views_backward_one_view_sampled_gradients(gpu_lib, mv):
    """The backward over all 64 views at full size, with a seeded image
    gradient on one seeded view and zero on the others: the summed gradients
    of 24 seeded primitives that view sees, drawn from every tile-count class
    (every attribute), against the oracle's exact windowed fp64 gradients of
    that view, element by element."""
    sc, cams, plan = mv
    rng = np.random.Generator(np.random.PCG64(4005))
    v = int(rng.integers(len(cams)))
    cam = cams[v]
    g_img = synth.random_dl_dimage(4006, (3, cam.height, cam.width))
    dl = torch.zeros_like(plan.image)
    off = 3 * plan.layout[v].pixel_offset
    dl[off:off + g_img.size] = torch.from_numpy(g_img.reshape(-1)).cuda()
    ds = plan.scenes[0]
    names = ("means", "scales", "quats", "opacities", "sh", "freqs", "weights")
    grads = {n: torch.zeros_like(getattr(ds, n)) for n in names}
    plan.backward(dl, [grads], accumulate=False)
    torch.cuda.synchronize()
    with torch.no_grad():
        pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    prims = stratified_primitives(pr, 4007, strata=((1, 1, 4), (2, 4, 6), (5, 9, 4), (10, 49, 6), (50, 400, 4)))
    assert len(prims) >= 20
    ref = O.primitive_grads_windowed(sc, cam, g_img, prims, pr_all=pr)
    n = sc.n
    gpu = {"means": grads["means"].cpu().numpy()[:, prims].T,
           "scales": grads["scales"].cpu().numpy()[:, prims].T,
           "quats": grads["quats"].cpu().numpy()[:, prims].T,
           "opacities": grads["opacities"].cpu().numpy()[prims],
           "sh": grads["sh"].cpu().numpy().reshape(n, 16, 3)[prims],
           "freqs": grads["freqs"].cpu().numpy().reshape(4, 3, n)[:, :, prims].transpose(2, 0, 1),
           "weights": grads["weights"].cpu().numpy()[:, prims].T}
    print(f"view {v}, tiles of the sample: {sorted(pr.tiles[prims].tolist())}")
    reports = check_sampled_grads(names, gpu, ref,
                                  lambda rows: O.primitive_grad_slack_windowed(sc, cam, g_img, prims[rows], pr_all=pr),
                                  f"view {v}")
    for name, rep in reports.items():
        print(name, rep)
