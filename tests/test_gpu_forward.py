"""GPU forward parity: preprocess (K1), binning (K2-K5) and blend (K6) against
the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import synth
from oracle import gabor_oracle as O

from gpu_helpers import assert_image, gpu_plan, last_ids_from_gpu, oracle_project, record_fields_np, assert_dispatch_order

pytestmark = pytest.mark.gpu


def _rel(a, b, floor):
    return np.abs(a - b) / (np.abs(b) + floor)


def test_preprocess_matches_oracle_1k_scene(gpu_lib):
    sc, cam = synth.scene_1k_k2_rgb(), synth.camera_128()
    ds, plan = gpu_plan(sc, [cam])
    plan.preprocess()
    torch.cuda.synchronize()
    pr = oracle_project(sc, cam)
    depth = plan.depth.cpu().numpy()[:sc.n]
    assert (depth.view(np.uint32) == pr.depth32.view(np.uint32)).all(), "depth keys must be bit-identical"
    tiles = plan.tiles_touched.cpu().numpy()[:sc.n]
    vis_g = tiles > 0
    vis_o = pr.visible.numpy()
    frag = pr.fragile_rect
    assert ((vis_g == vis_o) | frag).all()
    rect = plan.rect.cpu().numpy()[:sc.n].astype(np.int64)
    x0, y0, x1, y1 = rect[:, 0] & 0xFFFF, rect[:, 0] >> 16, rect[:, 1] & 0xFFFF, rect[:, 1] >> 16
    rg = np.stack([x0, y0, x1, y1], 1)
    sel = vis_o & vis_g & ~frag
    assert (rg[sel] == pr.rect[sel]).all()
    f = record_fields_np(plan)
    m = vis_o & vis_g & ~pr.fragile_prim
    np.testing.assert_allclose(f["mu2d"][m], pr.mu2d.numpy()[m], rtol=1e-5, atol=1e-4)
    con = pr.conic.numpy()[m]
    scale = np.abs(con).max(1, keepdims=True)
    assert (np.abs(f["conic"][m] - con) <= 1e-5 * scale + 1e-9).all()
    np.testing.assert_allclose(f["rgb"][m], pr.rgb.numpy()[m], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(f["opacity"][m], pr.opac.numpy()[m], rtol=1e-5)
    f2 = pr.f2d.numpy()[m]
    fs = np.abs(f2).max(axis=(1, 2), keepdims=True) + 1e-6
    assert (np.abs(f["f2d"][m] - f2) <= 1e-5 * fs).all(), np.abs(f["f2d"][m] - f2).max()


def _write_synthetic_geom(plan, rect, depth, vis):
    r = torch.zeros((plan.items, 2), dtype=torch.int64)
    rr = torch.from_numpy(rect.astype(np.int64))
    r[:, 0] = rr[:, 0] | (rr[:, 1] << 16)
    r[:, 1] = rr[:, 2] | (rr[:, 3] << 16)
    plan.rect.copy_(r.to(torch.int32).cuda())
    plan.depth.copy_(torch.from_numpy(depth).cuda())
    t = np.where(vis, (rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1]), 0).astype(np.int32)
    plan.tiles_touched.copy_(torch.from_numpy(t).cuda())


def _bin_sort_case(n, views, seed, width=200, height=150, hot_share=0.0, want_keys=True):
    sc = synth.uniform_scene(seed, n, 1)
    cams = [synth.pinhole_camera(width + 37 * v, height + 11 * v, 60.0, (0, 0, -3), (0, 0, 0)) for v in range(views)]
    # capacity for the largest rectangles (6 x 6 tiles) of every item
    ds, plan = gpu_plan(sc, cams, scene_of_view=[0] * views, capacity=36 * n * views + 1024, want_keys=want_keys)
    plan.preprocess()  # writes the view table
    rects, depths, viss = [], [], []
    for v, c in enumerate(cams):
        r, d, vi = synth.random_geom(100 * seed + v, n, c.tiles_x, c.tiles_y)
        if hot_share > 0:  # pile a share of the rectangles onto the first tiles
            hot = np.random.Generator(np.random.PCG64(seed + 77)).uniform(size=n) < hot_share
            r[hot, 0] = 0; r[hot, 1] = 0
            r[hot, 2] = 1 + (np.arange(n)[hot] % 2); r[hot, 3] = 1 + (np.arange(n)[hot] % 3 == 0)
            r[hot & ~vi] = 0
        rects.append(r); depths.append(d); viss.append(vi)
    rect, depth, vis = np.concatenate(rects), np.concatenate(depths), np.concatenate(viss)
    return cams, plan, rect, depth, vis


@pytest.mark.parametrize("n,views,seed,width,height,hot",
                         [(3000, 1, 1, 200, 150, 0.0), (20000, 2, 2, 200, 150, 0.0), (1, 1, 3, 200, 150, 0.0),
                          (9000, 3, 4, 200, 150, 0.0),
                          # a tile with ~11,000 pairs: sorted as runs of 1024 merged pairwise
                          (20000, 1, 5, 200, 150, 0.7),
                          # more than 8192 tiles take the radix-sort binning path; its tile passes
                          # use digits of 8 (38,859 tiles: 16 bits), 7 (13,005: 14 bits) and
                          # 6 bits (123,751: 17 bits)
                          (3000, 8, 6, 1024, 1024, 0.0), (2000, 3, 7, 1024, 1024, 0.0),
                          (800, 20, 8, 1024, 1024, 0.0)])
def test_bin_sort_bit_exact_on_synthetic_geometry(gpu_lib, n, views, seed, width, height, hot):
    """Stage-isolated K2-K5: seeded synthetic rects/depths (with ties) go into
    the GPU bin sort and the oracle's library stable sort; keys, values and
    ranges must be identical."""
    cams, plan, rect, depth, vis = _bin_sort_case(n, views, seed, width, height, hot)
    _write_synthetic_geom(plan, rect, depth, vis)
    plan.bin_sort()
    torch.cuda.synchronize()
    P = int(plan.num_pairs.item())
    assert int(plan.overflow.item()) == 0
    keys_o, vals_o, exp = _expected_bin_sort(cams, plan, rect, depth, vis, n)
    assert P == len(keys_o)
    kg = plan.keys.cpu().numpy()[:P].view(np.uint64)
    vg = plan.vals.cpu().numpy()[:P].view(np.uint32)
    assert (kg == keys_o).all()
    assert (vg == vals_o).all()
    rg = plan.ranges.cpu().numpy().view(np.uint32)
    assert (rg[:plan.tiles] == exp).all()


def _expected_bin_sort(cams, plan, rect, depth, vis, n):
    """The oracle's library stable sort of the synthetic pairs of every view:
    global keys, item ids and per-tile [start, end) ranges."""
    keys_o, vals_o = [], []
    for v, c in enumerate(cams):
        sl = slice(v * n, (v + 1) * n)
        k, vv, _ = O.bin_sort(rect[sl], depth[sl], vis[sl], c.tiles_x, c.num_tiles,
                              tile_offset=plan.layout[v].tile_offset, index_offset=v * n)
        keys_o.append(k); vals_o.append(vv)
    keys_o = np.concatenate(keys_o)
    vals_o = np.concatenate(vals_o)
    # global ranges: recompute from the oracle's global key order
    tl = (keys_o >> np.uint64(32)).astype(np.int64)
    exp = np.zeros((plan.tiles, 2), np.uint32)
    for t_ in np.unique(tl):
        idx = np.nonzero(tl == t_)[0]
        exp[t_] = (idx[0], idx[-1] + 1)
    return keys_o, vals_o, exp


@pytest.mark.parametrize("n,seed,hot", [(500, 11, 0.0), (3000, 12, 0.0), (9000, 13, 0.0), (20000, 14, 0.0),
                                        (20000, 15, 0.7)])
def test_blend_orders_the_lists_it_is_given_unsorted(gpu_lib, n, seed, hot):
    """Without keys the tile-count bin sort leaves every list of two or more
    pairs grouped but unordered, marked by bit 31 of its end, and sorts only
    the lists longer than 1024 itself; the forward blend orders the others
    (one wavefront up to 256 ids, quarters merged in LDS up to 1024) before
    blending them.  After the blend, vals and the ranges equal the oracle's
    stable sort exactly, for lists of every length class (500 items: tens of
    pairs per tile; 3000: hundreds; 9000: up to ~1000; 20000: beyond 1024;
    hot: one list of ~11,000)."""
    cams, plan, rect, depth, vis = _bin_sort_case(n, 1, seed, hot_share=hot, want_keys=False)
    _write_synthetic_geom(plan, rect, depth, vis)
    plan.bin_sort()
    torch.cuda.synchronize()
    P = int(plan.num_pairs.item())
    assert int(plan.overflow.item()) == 0
    keys_o, vals_o, exp = _expected_bin_sort(cams, plan, rect, depth, vis, n)
    assert P == len(keys_o)
    rg = plan.ranges.cpu().numpy().view(np.uint32)[:plan.tiles].copy()
    lens = exp[:, 1] - exp[:, 0]
    marked = (rg[:, 1] & 0x80000000) != 0
    # marked: exactly the lists of 2..1024 pairs; the bin sort ordered the longer ones
    assert (marked == ((lens >= 2) & (lens <= 1024))).all()
    assert (rg[:, 0] == exp[:, 0]).all() and ((rg[:, 1] & 0x7FFFFFFF) == exp[:, 1]).all()
    vg = plan.vals.cpu().numpy()[:P].view(np.uint32)
    long_ = lens > 1024
    for t_ in np.nonzero(long_)[0]:
        assert (vg[exp[t_, 0]:exp[t_, 1]] == vals_o[exp[t_, 0]:exp[t_, 1]]).all(), t_
    for t_ in np.nonzero(marked)[0]:  # the same ids, grouped by tile
        a, b = exp[t_]
        assert (np.sort(vg[a:b]) == np.sort(vals_o[a:b])).all(), t_
    print("lists", int(marked.sum()), "marked,", int(long_.sum()), "long; max", int(lens.max()))
    plan.render_fwd()
    torch.cuda.synchronize()
    vg = plan.vals.cpu().numpy()[:P].view(np.uint32)
    assert (vg == vals_o).all()
    assert (plan.ranges.cpu().numpy().view(np.uint32)[:plan.tiles] == exp).all()


def test_blend_list_sort_at_every_size_boundary(gpu_lib):
    """Lists of exactly the lengths where the list sort changes method (one
    wavefront with 1, 2 or 4 keys per lane up to 64, 128 and 256 ids; merged
    quarters of 2 and 4 keys per lane up to 512 and 1024; the bin sort's
    long-list kernel beyond) and one either side, with a fifth of the depths
    drawn from three values so that equal depths are ordered by item: after
    the blend every list equals the oracle's stable sort."""
    lens = [1, 2, 3, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2049]
    n = int(sum(lens))
    sc = synth.uniform_scene(16, n, 1)
    cam = synth.pinhole_camera(160, 48, 60.0, (0, 0, -3), (0, 0, 0))  # 10 x 3 tiles
    ds, plan = gpu_plan(sc, [cam], capacity=n + 1024)
    plan.preprocess()
    rng = np.random.Generator(np.random.PCG64(17))
    tile_of = np.repeat(np.arange(len(lens)), lens)
    rng.shuffle(tile_of)
    tx, ty = tile_of % cam.tiles_x, tile_of // cam.tiles_x
    rect = np.stack([tx, ty, tx + 1, ty + 1], 1).astype(np.int32)
    depth = rng.uniform(0.2, 50.0, size=n).astype(np.float32)
    ties = rng.uniform(size=n) < 0.2
    depth[ties] = rng.choice(np.array([1.0, 2.5, 7.25], np.float32), size=int(ties.sum()))
    vis = np.ones(n, bool)
    _write_synthetic_geom(plan, rect, depth, vis)
    plan.bin_sort()
    plan.render_fwd()
    torch.cuda.synchronize()
    assert int(plan.overflow.item()) == 0
    P = int(plan.num_pairs.item())
    keys_o, vals_o, exp = _expected_bin_sort([cam], plan, rect, depth, vis, n)
    assert P == n == len(vals_o)
    assert (plan.ranges.cpu().numpy().view(np.uint32)[:plan.tiles] == exp).all()
    vg = plan.vals.cpu().numpy()[:P].view(np.uint32)
    for t_ in range(len(lens)):
        a, b = exp[t_]
        assert b - a == lens[t_]
        assert (vg[a:b] == vals_o[a:b]).all(), (t_, lens[t_])


def test_unsorted_lists_render_exactly_like_sorted_ones(gpu_lib):
    """The 1000-primitive scene's K1 output binned with keys (every list sorted by the bin
    sort) and without (lists ordered by the blend): identical images, final
    transmittances, contributor counts, lists and ranges, bit for bit."""
    sc, cam = synth.scene_1k_k2_rgb(), synth.camera_128()
    outs = []
    for want_keys in (True, False):
        ds, plan = gpu_plan(sc, [cam], want_keys=want_keys)
        plan.forward()
        torch.cuda.synchronize()
        P = int(plan.num_pairs.item())
        outs.append((plan.image.cpu().numpy(), plan.final_T.cpu().numpy(), plan.n_contrib.cpu().numpy(),
                     plan.vals.cpu().numpy()[:P], plan.ranges.cpu().numpy()[:plan.tiles]))
    for a, b in zip(*outs):
        assert a.shape == b.shape and (a.view(np.uint32) == b.view(np.uint32)).all()


def test_bin_sort_end_to_end_1k_scene(gpu_lib):
    """K1 + K2-K5 on the 1000-primitive scene: the GPU's sorted keys equal the oracle's
    (no primitive of this scene sits within the rect tolerance of a tile
    boundary, so the comparison is exact)."""
    sc, cam = synth.scene_1k_k2_rgb(), synth.camera_128()
    ds, plan = gpu_plan(sc, [cam], want_keys=True)
    plan.preprocess()
    plan.bin_sort()
    torch.cuda.synchronize()
    pr = oracle_project(sc, cam)
    keys_o, vals_o, ranges_o = O.bin_sort(pr.rect, pr.depth32, pr.visible.numpy(), cam.tiles_x, cam.num_tiles)
    P = int(plan.num_pairs.item())
    kg = plan.keys.cpu().numpy()[:P].view(np.uint64)
    vg = plan.vals.cpu().numpy()[:P].view(np.uint32)
    if pr.fragile_rect.any():
        bad = set(np.nonzero(pr.fragile_rect)[0].tolist())
        keep_o = np.array([int(v) not in bad for v in vals_o])
        keep_g = np.array([int(v) not in bad for v in vg])
        kg, vg, keys_o, vals_o = kg[keep_g], vg[keep_g], keys_o[keep_o], vals_o[keep_o]
    else:
        assert (plan.ranges.cpu().numpy().view(np.uint32)[:cam.num_tiles] == ranges_o).all()
    assert (kg == keys_o).all() and (vg == vals_o).all()
    assert_dispatch_order(plan)


def test_render_forward_1k_scene(gpu_lib):
    sc, cam = synth.scene_1k_k2_rgb(), synth.camera_128()
    ds, plan = gpu_plan(sc, [cam])
    plan.forward()
    torch.cuda.synchronize()
    ref = O.render_scene(sc, cam, "binned")
    img = plan.view_image(0).cpu().numpy()
    assert_image(img, ref, "1k scene")
    T = plan.view_final_T(0).cpu().numpy()
    ok = ~ref.fragile
    assert np.abs(T - ref.final_T.numpy())[ok].max() <= 1e-4
    ids = last_ids_from_gpu(plan, 0)
    assert (ids[ok] == ref.last_id[ok]).all()


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (1.0, 0.5, 0.25)])
def test_render_forward_sh_and_background(gpu_lib, bg):
    sc = synth.uniform_scene(31, 3000, 4, sh_degree=3, log_scale_mu=-3.3)
    cam = synth.pinhole_camera(200, 136, 55.0, eye=(0.3, -0.2, -2.7), target=(0.0, 0.1, 0.0), bg=bg)
    ds, plan = gpu_plan(sc, [cam])
    plan.forward()
    ref = O.render_scene(sc, cam, "binned")
    assert_image(plan.view_image(0).cpu().numpy(), ref, f"sh3 K4 bg {bg}")


def test_render_forward_high_frequency(gpu_lib):
    """Frequencies scaled so that |f2d| reaches ~0.5 cycles/px."""
    sc = synth.uniform_scene(32, 2000, 3, sh_degree=-1, log_scale_mu=-2.8)
    sc.freqs *= 12.0
    cam = synth.camera_128()
    ds, plan = gpu_plan(sc, [cam])
    plan.forward()
    pr = oracle_project(sc, cam)
    print("max |f2d|", float(pr.f2d.norm(dim=-1).max()))
    ref = O.render_scene(sc, cam, "binned")
    assert_image(plan.view_image(0).cpu().numpy(), ref, "high frequency")


def test_render_forward_multiview_ragged(gpu_lib):
    """Several views of different (ragged, non-multiple-of-16) sizes in one
    launch per stage; each equals its own single-view oracle render."""
    sc = synth.uniform_scene(33, 1500, 2, sh_degree=1)
    cams = [synth.pinhole_camera(97, 61, 60.0, (0.0, 0.0, -3.0), (0, 0, 0)),
            synth.pinhole_camera(33, 130, 50.0, (1.0, 0.5, -2.5), (0, 0, 0), bg=(0.2, 0.2, 0.2)),
            synth.pinhole_camera(1, 1, 60.0, (0.0, 0.0, -3.0), (0, 0, 0)),
            synth.pinhole_camera(160, 17, 70.0, (-1.0, 0.0, -2.0), (0, 0, 0))]
    ds, plan = gpu_plan(sc, cams, scene_of_view=[0] * len(cams))
    plan.forward()
    for v, c in enumerate(cams):
        ref = O.render_scene(sc, c, "binned")
        assert_image(plan.view_image(v).cpu().numpy(), ref, f"view {v}")


def test_render_forward_empty_and_culled(gpu_lib):
    """All primitives behind the camera: background everywhere, no pairs."""
    sc = synth.uniform_scene(34, 500, 2, sh_degree=-1)
    sc.means[:, 2] = -5.0
    cam = synth.pinhole_camera(40, 40, 60.0, eye=(0.0, 0.0, -3.0), target=(0.0, 0.0, 0.0), bg=(0.3, 0.6, 0.9))
    ds, plan = gpu_plan(sc, [cam])
    plan.forward()
    assert int(plan.num_pairs.item()) == 0
    img = plan.view_image(0).cpu().numpy()
    np.testing.assert_array_equal(img, np.broadcast_to(np.array([0.3, 0.6, 0.9], np.float32)[:, None, None], img.shape))
    assert (plan.view_n_contrib(0).cpu().numpy() == 0).all()


def test_forward_is_deterministic(gpu_lib):
    sc, cam = synth.scene_1k_k2_rgb(), synth.camera_128()
    ds, plan = gpu_plan(sc, [cam])
    a = plan.forward().clone()
    b = plan.forward().clone()
    assert torch.equal(a, b)


def test_capacity_overflow_and_retry(gpu_lib):
    """A pair capacity that is too small sets the device flag; the plan grows
    its buffers and reaches the same image."""
    sc, cam = synth.scene_1k_k2_rgb(), synth.camera_128()
    ds, plan = gpu_plan(sc, [cam], capacity=100)
    plan.preprocess()
    plan.bin_sort()
    torch.cuda.synchronize()
    assert int(plan.overflow.item()) == 1
    assert int(plan.num_pairs.item()) > 100
    img = plan.forward().clone()
    assert plan.capacity > 100
    ds2, plan2 = gpu_plan(sc, [cam])
    assert torch.equal(img, plan2.forward())


def test_frequency_map_and_eval_counts(gpu_lib):
    """The analysis variant: frequency map against the oracle, and the image
    it renders is the same as the timed variant's."""
    sc = synth.uniform_scene(35, 2000, 3, sh_degree=1, log_scale_mu=-3.0)
    cam = synth.pinhole_camera(96, 64, 60.0, (0.2, 0.1, -3.0), (0, 0, 0))
    ds, plan = gpu_plan(sc, [cam])
    img = plan.forward().clone()
    fm = torch.zeros(96 * 64, dtype=torch.float32, device="cuda")
    cnt = torch.zeros((96 * 64, 2), dtype=torch.int32, device="cuda")
    plan.render_fwd(eval_counts=cnt, freq_map=fm)
    torch.cuda.synchronize()
    assert torch.equal(img, plan.image)
    ref = O.render_scene(sc, cam, "binned")
    ok = ~ref.fragile
    d = np.abs(fm.cpu().numpy().reshape(64, 96) - ref.freq_map.numpy())
    assert d[ok].max() <= 1e-4 * max(1.0, float(ref.freq_map.numpy().max()))
    c = cnt.cpu().numpy()
    ranges = plan.view_ranges(0).cpu().numpy().astype(np.int64)
    tile = (np.arange(64)[:, None] // 16) * 6 + (np.arange(96)[None, :] // 16)
    lens = (ranges[:, 1] - ranges[:, 0])[tile].reshape(-1)
    assert (c[:, 0] <= lens).all() and (c[:, 1] <= c[:, 0]).all()
    assert (c[:, 0] >= plan.view_n_contrib(0).cpu().numpy().reshape(-1)).all()


@pytest.mark.parametrize("k,deg", [(4, 3), (2, 1), (8, 0)])
def test_packed_rows_render_exactly_like_the_planes(gpu_lib, k, deg):
    """gabsplat_pack_rows writes each primitive's quaternion, frequencies and
    weights as one row (zeros after), and K1 reading those rows gives the
    records, depths, rects, tile counts and images of the planar input, bit
    for bit -- for one scene and for a batch of two scenes with rows."""
    from paper_2508_05343_amd.rasterize import DeviceScene, RenderPlan
    sc = synth.uniform_scene(90 + k, 3000, k, sh_degree=deg, log_scale_mu=-3.0)
    sc2 = synth.uniform_scene(190 + k, 2000, k, sh_degree=deg, log_scale_mu=-2.8)
    cam = synth.pinhole_camera(160, 120, 60.0, (0.1, 0.0, -3.0), (0, 0, 0))
    cam2 = synth.pinhole_camera(96, 80, 55.0, (-0.8, 0.3, -2.6), (0, 0, 0), bg=(0.3, 0.3, 0.3))
    ds, ds2 = DeviceScene.from_host(sc), DeviceScene.from_host(sc2)
    dr, dr2 = ds.with_rows(), ds2.with_rows()
    torch.cuda.synchronize()
    rs = gpu_lib.gabsplat_row_floats(k)
    rows = dr.rows.cpu().numpy()
    assert rows.shape == (sc.n, rs) and dr.rows.data_ptr() % 128 == 0
    assert np.array_equal(rows[:, 0:4], ds.quats.cpu().numpy().T)
    assert np.array_equal(rows[:, 4:4 + 3 * k], ds.freqs.cpu().numpy().T)
    assert np.array_equal(rows[:, 4 + 3 * k:4 + 4 * k], ds.weights.cpu().numpy().T)
    assert not rows[:, 4 + 4 * k:].any()
    for planar, packed, cams, sov in (([ds], [dr], [cam], None), ([ds, ds2], [dr, dr2], [cam, cam2, cam], [0, 1, 1])):
        a = RenderPlan(planar, cams, sov)
        b = RenderPlan(packed, cams, sov)
        a.forward()
        b.forward()
        torch.cuda.synchronize()
        for name in ("rec", "depth", "rect", "tiles_touched", "image", "final_T", "n_contrib"):
            x, y = getattr(a, name).cpu().numpy(), getattr(b, name).cpu().numpy()
            if name in ("rec", "depth", "rect"):  # rows of culled items are not written
                vis = a.tiles_touched.cpu().numpy()[:a.items] > 0
                x, y = x[:a.items][vis], y[:a.items][vis]
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), (name, len(cams))
