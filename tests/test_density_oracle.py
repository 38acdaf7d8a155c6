"""Pins of the density-control oracle (frequency-adaptive densification)."""
import numpy as np
import torch

import synth
from oracle import density_oracle as D
from oracle import gabor_oracle as O


def _stats(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    denom = rng.integers(0, 5, n).astype(np.float32)
    accum = (rng.exponential(0.0002, n) * denom).astype(np.float32)
    return accum, denom


def test_decisions_against_a_plain_loop():
    sc = synth.uniform_scene(5, 2000, 2, sh_degree=1, log_scale_mu=-4.6, log_scale_sigma=1.0)
    sc.opacities[::17] = 0.005
    accum, denom = _stats(sc.n, 6)
    prm = D.DensifyParams(scene_extent=1.0, prune_big=True, max_world_frac=0.05)
    kind = D.decide(sc, accum, denom, prm)
    for i in range(sc.n):
        avg = float(np.float32(accum[i] / denom[i])) if denom[i] > 0 else 0.0
        sm = float(max(sc.scales[i]))
        if sc.opacities[i] < np.float32(0.01) or sm > np.float32(0.05):
            exp = 3
        elif avg >= np.float32(0.0002):
            exp = 1 if sm <= np.float32(0.01) else 2
        else:
            exp = 0
        assert kind[i] == exp, i
    assert set(np.unique(kind)) == {0, 1, 2, 3}


def test_densify_counts_order_and_frequency_reset():
    sc = synth.uniform_scene(7, 1500, 3, sh_degree=-1, log_scale_mu=-4.6, log_scale_sigma=1.0)
    sc.opacities[::23] = 0.001
    accum, denom = _stats(sc.n, 8)
    prm = D.DensifyParams()
    rng = np.random.Generator(np.random.PCG64(9))
    normals = rng.normal(size=(sc.n, 2, 3)).astype(np.float32)
    kind = D.decide(sc, accum, denom, prm)
    out, src, tag = D.densify(sc, accum, denom, normals, prm)
    nk, nc, ns = (kind == 0).sum(), (kind == 1).sum(), (kind == 2).sum()
    assert len(src) == nk + 2 * nc + 2 * ns
    assert (np.diff(src[:nk + nc]) > 0).all()
    # originals keep every attribute, children have f = 0.001 and w = 0.01 everywhere
    orig = tag == 0
    np.testing.assert_array_equal(out["freqs"][orig], sc.freqs[src[orig]])
    assert (out["freqs"][~orig] == 0.001).all() and (out["weights"][~orig] == 0.01).all()
    # clones keep position and scale; split children shrink by 1.6
    cl = tag == 1
    np.testing.assert_array_equal(out["means"][cl], sc.means[src[cl]])
    sp = tag >= 2
    np.testing.assert_allclose(out["scales"][sp], sc.scales[src[sp]] / 1.6, rtol=1e-7)
    # pruned primitives leave nothing behind
    assert not np.isin(src, np.nonzero(kind == 3)[0]).any()


def test_split_children_are_drawn_from_the_parent_gaussian():
    """Child offsets R(q)(s * z), z ~ N(0, I), have covariance R S S^T R^T,
    the parent's covariance (Sec. 3.1)."""
    sc = synth.uniform_scene(10, 1, 1, sh_degree=-1)
    sc.scales[0] = [0.3, 0.1, 0.05]
    rng = np.random.Generator(np.random.PCG64(11))
    m = 200000
    big = sc.subset(np.zeros(m, np.int64))
    accum = np.ones(m, np.float32)
    denom = np.ones(m, np.float32)
    normals = rng.normal(size=(m, 2, 3))
    out, src, tag = D.densify(big, accum, denom, normals, D.DensifyParams(percent_dense=0.01))
    off = out["means"] - big.means[src].astype(np.float64)
    cov = np.cov(off.T)
    Sig = O.covariance_3d(torch.tensor(sc.scales.astype(np.float64)),
                          torch.tensor(sc.quats.astype(np.float64))).numpy()[0]
    np.testing.assert_allclose(cov, Sig, atol=4e-4)


def test_stats_in_ndc_units():
    g = np.array([[1.0, 0.0], [0.0, 2.0], [3.0, 4.0]])
    acc = np.zeros(3)
    den = np.zeros(3)
    D.accumulate_stats(g, np.array([True, True, False]), 200, 100, acc, den)
    np.testing.assert_allclose(acc, [100.0, 100.0, 0.0])
    np.testing.assert_array_equal(den, [1, 1, 0])


def test_periodic_reset():
    sc = synth.uniform_scene(12, 50, 2)
    w, o = D.periodic_reset(sc)
    assert (w == 0.01).all() and (o <= 0.02).all()
    assert (o == np.minimum(sc.opacities.astype(np.float64), 0.02)).all()


def test_decision_boundaries_from_the_text():
    """The three thresholds at their exact boundary values, with the expected
    decision written from the rule the paper adopts (Sec. 3.4.2 densifies as
    3DGS does; supplementary B gives the prune threshold): a primitive is
    selected when its mean view-space gradient is AT LEAST the threshold,
    cloned when its largest scale is AT MOST percent_dense * extent (split when
    larger), and pruned when its opacity is BELOW min_opacity.  Values one
    float32 step to either side flip the decision.  A '>' for '>=', a '<' for
    '<=' or a '<=' for '<' fails one of the rows."""
    f32 = np.float32
    thr, pd, ext, mo = f32(2e-4), f32(0.01), f32(1.0), f32(0.01)
    below = lambda x: np.nextafter(f32(x), f32(0))  # noqa: E731
    above = lambda x: np.nextafter(f32(x), f32(1))  # noqa: E731
    small, big = f32(0.005), f32(0.02)
    # (mean gradient, max scale, opacity) -> expected kind (0 keep, 1 clone, 2 split, 3 prune)
    rows = [
        (thr, small, f32(0.5), 1),           # gradient exactly at the threshold: selected
        (below(thr), small, f32(0.5), 0),    # just below: kept
        (thr, pd * ext, f32(0.5), 1),        # max scale exactly percent_dense * extent: clone
        (thr, above(pd * ext), f32(0.5), 2),  # just above: split
        (thr, big, f32(0.5), 2),
        (below(thr), big, f32(0.5), 0),
        (f32(0.0), small, mo, 0),            # opacity exactly min_opacity: not pruned
        (f32(0.0), small, below(mo), 3),     # just below: pruned
        (thr, small, below(mo), 3),          # pruning wins over cloning
        (thr, big, below(mo), 3),            # and over splitting
    ]
    n = len(rows)
    sc = synth.uniform_scene(11, n, 2, sh_degree=-1)
    sc.scales[:] = f32(0.001)
    for i, (g, s, o, _) in enumerate(rows):
        sc.scales[i, i % 3] = s          # the largest scale on a varying axis
        sc.opacities[i] = o
    denom = np.ones(n, np.float32)
    accum = np.array([r[0] for r in rows], np.float32)
    prm = D.DensifyParams(grad_threshold=2e-4, percent_dense=0.01, scene_extent=1.0, min_opacity=0.01)
    kind = D.decide(sc, accum, denom, prm)
    assert kind.tolist() == [r[3] for r in rows]
    # a mean over several views: accum / denom at the threshold is still selected
    sc2 = sc.subset(np.array([0]))
    assert D.decide(sc2, np.array([f32(thr) * f32(4.0)], np.float32), np.array([4.0], np.float32), prm).tolist() == [1]
    # never seen (denom 0): mean gradient 0, kept
    assert D.decide(sc2, np.array([f32(1.0)], np.float32), np.array([0.0], np.float32), prm).tolist() == [0]
