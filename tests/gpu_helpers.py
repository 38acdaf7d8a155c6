"""Shared helpers of the GPU parity tests (inputs come from the seeded
generators, expected values from the CPU oracle only)."""
import numpy as np
import torch

import synth
from oracle import gabor_oracle as O


def gpu_plan(scenes, cams, scene_of_view=None, want_keys=True, capacity=None):
    from paper_2508_05343_amd.rasterize import DeviceScene, RenderPlan
    if not isinstance(scenes, (list, tuple)):
        scenes = [scenes]
    ds = [DeviceScene.from_host(s) for s in scenes]
    plan = RenderPlan(ds, cams, scene_of_view, pair_capacity=capacity, want_keys=want_keys)
    return ds, plan


def record_fields_np(plan):
    return {k: v.detach().cpu().numpy() for k, v in plan.record_fields().items()}


def oracle_project(scene, cam):
    with torch.no_grad():
        return O.project(O.scene_tensors(scene), O.camera_tensors(cam), scene)


def last_ids_from_gpu(plan, v, n_items_offset=0):
    """Primitive id of the last blended primitive per pixel (-1 if none) from
    the GPU's n_contrib (a position in the tile's sorted list)."""
    c = plan.cams[v]
    H, W = c.height, c.width
    nc = plan.view_n_contrib(v).cpu().numpy().astype(np.int64)
    ranges = plan.view_ranges(v).cpu().numpy().astype(np.int64)
    vals = plan.vals.cpu().numpy().astype(np.int64)
    tx = (np.arange(W) // 16)[None, :]
    ty = (np.arange(H) // 16)[:, None]
    tile = ty * ((W + 15) // 16) + tx
    start = ranges[tile, 0]
    pos = start + nc - 1
    ids = np.where(nc > 0, vals[np.clip(pos, 0, len(vals) - 1)], -1)
    off = plan.layout[v].item_offset
    return np.where(ids >= 0, ids - off, -1)


def compare_image(gpu_img, ref, atol=1e-4):
    """Max abs error on non-fragile pixels, fragile fraction, and the count of
    non-fragile pixels above atol."""
    d = np.abs(gpu_img - ref.color.numpy())
    valid = ~np.isnan(ref.color.numpy()[0])
    ok = valid & ~ref.fragile
    bad = (d.max(0) > atol) & ok
    return float(d[:, ok].max()) if ok.any() else 0.0, float(ref.fragile[valid].mean()), int(bad.sum())
