"""The oracle's exact gradients at the size of the training-step workload
(1,000,000 primitives, K = 4, SH degree 3, 1297x840), pinned by fp64 central
finite differences of its own forward.  Perturbing one primitive only changes
the pixels of the tiles in its rectangle (outside them its alpha is below
1/255), so each difference re-renders only that window.  The primitives are
a seeded part of the subset whose GPU gradients are checked against the
oracle's (one of every size class, the largest included)."""
import numpy as np
import pytest
import torch

import synth
from oracle import gabor_oracle as O

from sampling import stratified_primitives

ATTRS = ("means", "scales", "quats", "opacities", "sh", "freqs", "weights")
# finite-difference steps: small enough that no pixel decision (alpha against
# 1/255, the stop rule) is crossed, large enough that rounding stays below
# the tolerance (scales: relative step)
STEP = dict(means=1e-6, scales=1e-6, quats=1e-6, opacities=1e-6, sh=1e-5, freqs=1e-5, weights=1e-6)


@pytest.fixture(scope="module")
def frame():
    sc, cam = synth.scene_1m_k4_sh3(), synth.camera_1297x840()
    with torch.no_grad():
        pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    g_img = synth.random_dl_dimage(1003, (3, cam.height, cam.width))
    return sc, cam, pr, g_img


def _fd_entries(sc, i, full):
    """(attribute, flat index) pairs to perturb: every scalar of the geometry,
    frequencies and weights, and four SH coefficients (colour is linear in
    them); for a large primitive the means, scales, opacity and the first
    component's frequency and weight."""
    if not full:
        return [("means", 0), ("means", 1), ("scales", 0), ("opacities", 0), ("freqs", 0), ("weights", 0)]
    ent = [(a, j) for a in ("means", "scales", "quats", "freqs", "weights")
           for j in range(int(np.asarray(getattr(sc, a)[i]).size))]
    ent.append(("opacities", 0))
    ent += [("sh", j) for j in (0, 5, 22, 47)]
    return ent


def test_windowed_gradients_match_finite_differences_at_full_size(frame):
    sc, cam, pr, g_img = frame
    sample = stratified_primitives(pr, 3003)
    tiles = pr.tiles[sample]
    # one primitive of every size class, up to 120 tiles
    picks = []
    for lo, hi in ((1, 1), (2, 4), (5, 9), (10, 49), (50, 80)):
        c = sample[(tiles >= lo) & (tiles <= hi)]
        if len(c):
            picks.append(int(c[0]))
    assert len(picks) == 5 and pr.tiles[picks[-1]] >= 50
    ref = O.primitive_grads_windowed(sc, cam, g_img, picks, pr_all=pr)
    order = O.depth_order(pr.depth32, pr.visible.numpy())
    for i, gr in zip(picks, ref):
        win = O.window_setup(pr, order, i)
        base = {a: np.asarray(getattr(sc, a)[i], np.float64).copy() for a in ATTRS}
        gmax = max(float(np.abs(gr[a]).max()) for a in ATTRS)
        assert gmax > 0
        for a, j in _fd_entries(sc, i, pr.tiles[i] < 50):
            x = base[a].reshape(-1)
            ad = float(np.asarray(gr[a]).reshape(-1)[j])
            h = STEP[a] * (abs(float(x[j])) if a == "scales" else 1.0)
            for _ in range(4):
                f = {}
                for m in (2, 1, -1, -2):
                    att = {k: v.copy() for k, v in base.items()}
                    att[a].reshape(-1)[j] = x[j] + m * h
                    f[m] = O.primitive_loss_windowed(sc, cam, g_img, i, att, pr_all=pr, win=win)
                roundoff = 3e-14 * max(abs(v) for v in f.values()) / h
                tol = 1e-6 * abs(ad) + 1e-8 * gmax + roundoff
                d1, d2 = (f[1] - f[-1]) / (2.0 * h), (f[2] - f[-2]) / (4.0 * h)
                # the forward is piecewise smooth: a pixel decision (alpha
                # against 1/255, the stop rule) crossed inside the stencil
                # shows as disagreeing one- and two-step differences; take a
                # smaller stencil then
                if abs(d1 - d2) <= tol:
                    break
                h /= 7.0
            else:
                pytest.fail(f"no smooth stencil for primitive {i}, {a}[{j}]")
            # five-point central difference: truncation error O(h^4)
            fd = (8.0 * (f[1] - f[-1]) - (f[2] - f[-2])) / (12.0 * h)
            assert abs(fd - ad) <= tol, (i, int(pr.tiles[i]), a, j, fd, ad)
