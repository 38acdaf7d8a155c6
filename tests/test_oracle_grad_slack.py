"""Pins of the oracle's gradient slack (the jump of the exact gradient when a
decision taken within rounding of its threshold goes the other way).

The slack is computed by flipping the decision inside the blend.  Here the
other branch is reached the way a float32 rasterizer reaches it: by moving an
input by one float32 step across the threshold, rendering again and
differentiating again.  The difference of the two exact gradients must be the
slack, element by element (the one-ulp input change moves the smooth part of
the gradient by ~1e-7 relative only)."""
import numpy as np
import pytest
import torch

import synth
from oracle import gabor_oracle as O

from test_oracle_pins import axis_camera, make_scene


def _alpha_at(scene, cam, i, px, py):
    """alpha_i (before the clamp) at the centre of pixel (px, py), fp64."""
    pr = O.project(O.scene_tensors(scene), O.camera_tensors(cam), scene)
    res = O.blend_pixels(pr, np.array([i]), torch.tensor([px + 0.5], dtype=O.DT),
                         torch.tensor([py + 0.5], dtype=O.DT), O.camera_tensors(cam)["bg"])
    # with one candidate alone: colour = alpha c + (1 - alpha) bg; solve for alpha from T
    return 1.0 - float(res.final_T[0]) if res.n_blended[0] else None


def _with_opacity(scene, i, o32):
    op = scene.opacities.copy()
    op[i] = o32
    return synth.Scene(means=scene.means, scales=scene.scales, quats=scene.quats, opacities=op,
                       freqs=scene.freqs, weights=scene.weights, colors=scene.colors, sh=scene.sh)


def _bracket(scene, i, side_is_hi, lo, hi, iters=80):
    """Bisect the float32 opacity of primitive i between lo and hi (float32)
    for the two neighbouring float32 values where ``side_is_hi(scene)``
    changes from False to True."""
    lo, hi = np.float32(lo), np.float32(hi)
    for _ in range(iters):
        if np.nextafter(lo, np.float32(1)) >= hi:
            break
        mid = np.float32((np.float64(lo) + np.float64(hi)) / 2)
        if mid <= lo or mid >= hi:
            break
        if side_is_hi(_with_opacity(scene, i, mid)):
            hi = mid
        else:
            lo = mid
    return lo, hi


def _compare_jump(s_lo, s_hi, cam, g):
    """The slack of each side equals the jump between the two sides' exact
    gradients."""
    g_lo = O.render_grads(s_lo, cam, g, "binned")
    g_hi = O.render_grads(s_hi, cam, g, "binned")
    for s in (s_lo, s_hi):
        sl = O.render_grad_slack(s, cam, g)
        for name in g_lo:
            if g_lo[name].size == 0:
                continue
            jump = np.abs(g_hi[name] - g_lo[name])
            scale = max(np.abs(g_lo[name]).max(), 1e-30)
            np.testing.assert_allclose(sl[name], jump, rtol=2e-3, atol=2e-6 * scale, err_msg=name)
    return g_lo, g_hi


def test_slack_of_a_skip_decision_equals_the_jump_across_the_threshold():
    """Primitive 1 (behind primitive 0, Gabor components on) reaches pixel
    (20, 14) with alpha at 1/255: the float32 opacities on either side of the
    point where that alpha crosses 1/255 give two exact gradients whose
    difference is the slack of the flipped skip decision."""
    cam = axis_camera(W=40, H=32, f=40.0, bg=(0.2, 0.1, 0.3))
    means = [[0.02, -0.01, 2.0], [-0.06, -0.03, 2.5]]
    scales = [[0.05, 0.07, 0.05], [0.06, 0.04, 0.05]]
    quats = [[1.0, 0.1, -0.2, 0.05], [0.9, -0.1, 0.3, 0.2]]
    freqs = [[[1.5, -0.7, 0.4], [-0.3, 2.0, 0.1]], [[0.8, 0.9, -0.5], [2.2, -1.0, 0.3]]]
    weights = [[0.2, 0.15], [0.25, 0.1]]
    colors = [[0.9, 0.2, 0.1], [0.1, 0.7, 0.8]]
    base = make_scene(means, scales, quats, [0.6, 0.5], colors, freqs, weights)
    px, py, i = 20, 14, 1
    a0 = _alpha_at(base, cam, i, px, py)
    assert a0 is not None and a0 > 0.02
    # opacity that puts alpha_1 at (20, 14) on 1/255 (alpha is linear in o)
    o_star = 0.5 * O.ALPHA_MIN / a0
    lo, hi = _bracket(base, i, lambda s: (_alpha_at(s, cam, i, px, py) or 0.0) >= O.ALPHA_MIN,
                      o_star * (1 - 1e-5), o_star * (1 + 1e-5))
    s_lo, s_hi = _with_opacity(base, i, lo), _with_opacity(base, i, hi)
    img_hi = O.render_scene(s_hi, cam, "binned")
    img_lo = O.render_scene(s_lo, cam, "binned")
    # exactly one decision is fragile, and it is this one
    assert int(img_hi.n_fragile.sum()) == 1 and bool(img_hi.fragile[py, px])
    assert int(img_lo.n_fragile.sum()) == 1 and bool(img_lo.fragile[py, px])
    assert img_hi.n_blended[py, px] == img_lo.n_blended[py, px] + 1
    g = synth.random_dl_dimage(31, (3, cam.height, cam.width))
    g_lo, g_hi = _compare_jump(s_lo, s_hi, cam, g)
    # the jump is real: it exceeds the relative bound on primitive 1's mean
    d = np.abs(g_hi["means"][1] - g_lo["means"][1])
    assert (d > 1e-3 * np.abs(g_lo["means"][1])).any()


def test_slack_of_a_stop_decision_equals_the_jump_across_the_threshold():
    """The termination stack (three primitives of opacity 0.95 centred on
    pixel (8, 8)) with a fourth whose opacity puts T (1 - alpha) on 1e-4: the
    float32 opacities on either side of the stop give two exact gradients whose
    difference is the slack of the flipped stop decision."""
    cam = axis_camera(W=16, H=16, f=16.0, bg=(0.25, 0.5, 0.75))
    depths = [1.0, 2.0, 3.0, 4.0]
    colors = [[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [0.6, 0.3, 0.9]]
    base = make_scene([[z / 32, z / 32, z] for z in depths], [[0.05] * 3] * 4, [[1, 0, 0, 0]] * 4,
                      [0.95, 0.95, 0.95, 0.2], colors)
    px = py = 8

    def stops(s):
        img = O.render_scene(s, cam, "binned")
        return img.n_blended[py, px] == 3
    lo, hi = _bracket(base, 3, stops, 0.19, 0.21)
    s_lo, s_hi = _with_opacity(base, 3, lo), _with_opacity(base, 3, hi)
    img_hi = O.render_scene(s_hi, cam, "binned")
    img_lo = O.render_scene(s_lo, cam, "binned")
    assert img_hi.n_blended[py, px] == 3 and img_lo.n_blended[py, px] == 4
    assert int(img_hi.n_fragile.sum()) == 1 and int(img_lo.n_fragile.sum()) == 1
    g = synth.random_dl_dimage(32, (3, cam.height, cam.width))
    _compare_jump(s_lo, s_hi, cam, g)


def test_slack_is_zero_without_fragile_decisions_and_windowed_equals_full():
    """No fragile decision, no slack; the windowed slack of a primitive is
    its row of the whole-image slack."""
    from test_oracle_pins import tiny_scene
    sc = tiny_scene(41, n=14, k=2)
    cam = axis_camera()
    g = synth.random_dl_dimage(33, (3, cam.height, cam.width))
    img = O.render_scene(sc, cam, "binned")
    full = O.render_grad_slack(sc, cam, g)
    if int(img.n_fragile.sum()) == 0:
        assert all(float(np.abs(v).max()) == 0.0 for v in full.values())
    # a scene with a fragile skip decision: reuse the skip-decision construction
    cam2 = axis_camera(W=40, H=32, f=40.0, bg=(0.2, 0.1, 0.3))
    base = make_scene([[0.02, -0.01, 2.0], [-0.06, -0.03, 2.5]], [[0.05, 0.07, 0.05], [0.06, 0.04, 0.05]],
                      [[1.0, 0.1, -0.2, 0.05], [0.9, -0.1, 0.3, 0.2]], [0.6, 0.5], [[0.9, 0.2, 0.1], [0.1, 0.7, 0.8]],
                      [[[1.5, -0.7, 0.4], [-0.3, 2.0, 0.1]], [[0.8, 0.9, -0.5], [2.2, -1.0, 0.3]]],
                      [[0.2, 0.15], [0.25, 0.1]])
    a0 = _alpha_at(base, cam2, 1, 20, 14)
    s = _with_opacity(base, 1, np.float32(0.5 * O.ALPHA_MIN / a0))
    assert int(O.render_scene(s, cam2, "binned").n_fragile.sum()) >= 1
    g2 = synth.random_dl_dimage(34, (3, cam2.height, cam2.width))
    full = O.render_grad_slack(s, cam2, g2)
    assert float(np.abs(full["means"]).max()) > 0.0
    win = O.primitive_grad_slack_windowed(s, cam2, g2, [0, 1])
    for i in (0, 1):
        for name, v in win[i].items():
            np.testing.assert_allclose(v, full[name][i], rtol=1e-10, atol=1e-300, err_msg=f"{name}[{i}]")
