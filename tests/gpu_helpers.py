"""Shared helpers of the GPU parity tests (inputs come from the seeded
generators, expected values from the CPU oracle only)."""
import numpy as np
import torch

import synth
from oracle import gabor_oracle as O


def gpu_plan(scenes, cams, scene_of_view=None, want_keys=False, capacity=None):
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


# Largest fraction of fragile pixels a forward comparison accepts (pixels
# where some decision of the oracle lies within its tolerance of a threshold).
MAX_FRAGILE_FRACTION = 0.01


def compare_image(gpu_img, ref, atol=1e-4):
    """Compares a rendered [3,H,W] image with the oracle's over the pixels the
    oracle rendered.  Non-fragile pixels must be within ``atol``; a fragile
    pixel within atol + fragile_bound * colour_span, the largest change its
    fragile decisions can cause (each alpha near 1/255 at most 2 alpha T span,
    each stop-rule decision near 1e-4 at most T span, T the transmittance
    before it).  Returns (max error on non-fragile pixels, fragile fraction,
    number of pixels outside their bound)."""
    c = ref.color.numpy()
    d = np.abs(gpu_img - c).max(0)
    valid = ~np.isnan(c[0])
    bound = atol + ref.fragile_bound * ref.colour_span
    bad = valid & ~(d <= bound)
    ok = valid & ~ref.fragile
    err = float(d[ok].max()) if ok.any() else 0.0
    frac = float(ref.fragile[valid].mean()) if valid.any() else 0.0
    return err, frac, int(bad.sum())


def assert_image(gpu_img, ref, label="", atol=1e-4, max_fragile=MAX_FRAGILE_FRACTION):
    """compare_image, asserted: every pixel inside its bound and at most
    ``max_fragile`` of the pixels fragile."""
    err, frac, nbad = compare_image(gpu_img, ref, atol)
    print(f"{label}: max err {err:.3e} (non-fragile), fragile {frac:.4%}, outside bound {nbad}")
    assert nbad == 0, (label, nbad, err)
    assert err <= atol, (label, err)
    assert frac <= max_fragile, (label, frac)
    return err, frac


def check_grads_elementwise(name, gpu, ref, slack=None, rel=1e-3, floor=1e-3, max_outlier_frac=1e-3,
                            norm_tol=1e-3):
    """Gradient parity per element: |g - g_ref| <= rel (|g_ref| + floor max|g_ref|)
    + slack for all but at most max_outlier_frac of the elements (rounded
    down), and the pooled relative L2 error below norm_tol.  ``slack`` (the
    oracle's render_grad_slack / primitive_grad_slack_windowed, same shape as
    ref) is the summed gradient jump of the decisions taken within rounding of
    their thresholds, which a float32 rasterizer may take either way; the L2
    check allows it too.  Returns (outliers, worst ratio of error to bound,
    relative L2 error, elements with slack)."""
    g = np.asarray(gpu, np.float64).reshape(-1)
    r = np.asarray(ref, np.float64).reshape(-1)
    sl = np.zeros_like(r) if slack is None else np.asarray(slack, np.float64).reshape(-1)
    assert g.shape == r.shape == sl.shape, (name, g.shape, r.shape, sl.shape)
    scale = np.abs(r).max() if r.size else 0.0
    bound = rel * (np.abs(r) + floor * scale) + sl
    err = np.abs(g - r)
    out = ~(err <= bound) if scale > 0 else ~(err <= sl)
    nout = int(out.sum())
    allowed = int(max_outlier_frac * r.size)
    worst = float((err / np.maximum(bound, 1e-300)).max()) if r.size else 0.0
    nrm = max(np.linalg.norm(r), 1e-30)
    l2 = float(np.linalg.norm(g - r) / nrm)
    l2_slack = float(np.linalg.norm(sl) / nrm)
    if nout:
        j = int(np.argmax(err / np.maximum(bound, 1e-300)))
        print(f"  {name}: {nout}/{r.size} outside the bound (allowed {allowed}); worst at {j}: "
              f"gpu {g[j]:.6e} ref {r[j]:.6e} slack {sl[j]:.3e}")
    assert nout <= allowed, (name, nout, allowed, worst)
    assert l2 <= norm_tol + l2_slack, (name, l2, l2_slack)
    return nout, worst, l2, int((sl > 0).sum())


def check_sampled_grads(names, gpu, ref_rows, slack_rows, label=""):
    """Element-wise parity of the gradients of sampled primitives.
    ``gpu[name]`` holds one row per sampled primitive, ``ref_rows`` the
    oracle's per-primitive gradient dicts (primitive_grads_windowed), and
    ``slack_rows(rows)`` returns the oracle's slack dicts of the listed rows
    (primitive_grad_slack_windowed).  An element inside the plain bound is
    inside bound + slack too, so the slack is only evaluated for the
    primitives with an element outside the plain bound.  Returns the
    per-attribute reports of check_grads_elementwise."""
    m = len(ref_rows)
    ref = {n: np.stack([r[n] for r in ref_rows]) for n in names}
    need = set()
    for n in names:
        r = ref[n].reshape(m, -1)
        g = np.asarray(gpu[n], np.float64).reshape(r.shape)
        scale = np.abs(r).max() if r.size else 0.0
        out = ~(np.abs(g - r) <= 1e-3 * (np.abs(r) + 1e-3 * scale))
        need |= set(np.nonzero(out.any(1))[0].tolist())
    slack = {n: np.zeros_like(ref[n]) for n in names}
    if need:
        rows = sorted(need)
        for j, d in zip(rows, slack_rows(rows)):
            for n in names:
                slack[n][j] = d[n]
    print(f"{label}: slack evaluated for {len(need)} of {m} primitives")
    return {n: check_grads_elementwise(f"{label} {n}", np.asarray(gpu[n]).reshape(ref[n].shape), ref[n], slack[n])
            for n in names}


def order_bucket(lengths):
    """Dispatch bucket of a tile list length: 0 for an empty list, else
    1 + 8 floor(log2 L) + the three bits of L after its leading one (capped at
    159), i.e. geometric buckets 2^(1/8) apart."""
    L = np.asarray(lengths, np.int64)
    out = np.zeros(L.shape, np.int64)
    nz = L > 0
    # exact bit length (log2 rounding cannot be trusted at powers of two)
    lz = np.array([int(x).bit_length() - 1 if x > 0 else 0 for x in L.ravel()], np.int64).reshape(L.shape)
    frac = np.where(lz >= 3, (L >> np.maximum(lz - 3, 0)) & 7, (L << np.maximum(3 - lz, 0)) & 7)
    out[nz] = np.minimum(1 + 8 * lz[nz] + frac[nz], 159)
    return out


def assert_dispatch_order(plan):
    """The blend's dispatch order after the ranges: a permutation of the tile
    ids whose list-length buckets never increase."""
    T = plan.tiles
    buf = plan.ranges_buf.cpu().numpy().view(np.uint32).astype(np.int64)
    ranges, order = buf[:2 * T].reshape(T, 2), buf[2 * T:3 * T]
    assert np.array_equal(np.sort(order), np.arange(T))
    b = order_bucket(ranges[:, 1] - ranges[:, 0])[order]
    assert (np.diff(b) <= 0).all()
