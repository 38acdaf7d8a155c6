"""CPU reference for frequency-adaptive density control (test infrastructure
only; shares no code with the GPU path).

Sec. 3.4.2: primitives whose accumulated view-space positional gradient
exceeds a threshold are densified (cloned when small, split when large) as in
3DGS, and -- the paper's change -- the frequencies and frequency weights of
every newly generated child are reset to small values; every few thousand
iterations all frequency weights are reset together with the opacity reset.
Small values follow the paper's initialisation (f = 0.001, w = 0.01, Sec.
3.4.1 and Sec. 4 implementation details; supplementary B: reset to 0.001 and
0.01 after densification, prune threshold 0.01, opacity reset 0.02).

The AbsGS variant (the densification the paper plugs its primitive into in
Sec. 4.1 / Table 1) adds a second statistic, the homodirectional gradient:
the per-axis sums over pixels of the absolute per-pixel mean gradients, in
the same NDC units.  Reading: it widens the split test only -- a large
primitive splits when either statistic reaches its threshold; cloning keeps
the ordinary statistic.

Everything here is plain numpy in float64 on float32 inputs; decisions
(comparisons against thresholds) are taken on the float32 values.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class DensifyParams:
    grad_threshold: float = 0.0002   # on the mean view-space (NDC) positional gradient norm
    percent_dense: float = 0.01      # clone if max scale <= percent_dense * extent, else split
    scene_extent: float = 1.0
    min_opacity: float = 0.01        # prune below
    max_world_frac: float = 0.1      # prune if max scale > max_world_frac * extent (when prune_big)
    prune_big: bool = False
    freq_reset: float = 0.001        # every axis of every frequency of a new child
    weight_reset: float = 0.01       # every frequency weight of a new child
    split_count: int = 2
    split_shrink: float = 1.0 / 1.6  # child scale factor (3DGS: 1 / (0.8 N))
    abs_grad_threshold: float = 0.0  # AbsGS split threshold on the homodirectional statistic (0: off)


def _ndc_norm(g, width, height):
    g = np.asarray(g, np.float64)
    return np.sqrt((g[:, 0] * width / 2.0) ** 2 + (g[:, 1] * height / 2.0) ** 2)


def accumulate_stats(grad_mu2d: np.ndarray, visible: np.ndarray, width: int, height: int,
                     accum: np.ndarray, denom: np.ndarray, abs_mu2d=None, accum_abs=None):
    """accum += |dL/d mu2d| measured in normalised device coordinates
    (pixel gradient times (W/2, H/2)), denom += 1, for the visible primitives;
    with abs_mu2d (per-axis sums of |dL_p/d mu2d| over pixels) also
    accum_abs += its norm in the same units."""
    v = np.asarray(visible, bool)
    accum[v] += _ndc_norm(grad_mu2d, width, height)[v]
    denom[v] += 1.0
    if abs_mu2d is not None:
        accum_abs[v] += _ndc_norm(abs_mu2d, width, height)[v]


def quat_rot(q):
    q = np.asarray(q, np.float64)
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _mean(accum, denom):
    accum = np.asarray(accum, np.float32)
    return np.where(denom > 0, accum / np.where(denom > 0, denom, 1), 0).astype(np.float32)


def decide(scene, accum, denom, prm: DensifyParams, accum_abs=None):
    """Per primitive: 0 keep, 1 clone, 2 split, 3 prune."""
    denom = np.asarray(denom, np.float32)
    avg = _mean(accum, denom)
    smax = np.asarray(scene.scales, np.float32).max(1)
    sel = avg >= np.float32(prm.grad_threshold)
    sel_split = sel
    if prm.abs_grad_threshold > 0:
        sel_split = sel | (_mean(accum_abs, denom) >= np.float32(prm.abs_grad_threshold))
    big = smax > np.float32(prm.percent_dense) * np.float32(prm.scene_extent)
    prune = np.asarray(scene.opacities, np.float32) < np.float32(prm.min_opacity)
    if prm.prune_big:
        prune |= smax > np.float32(prm.max_world_frac) * np.float32(prm.scene_extent)
    kind = np.zeros(scene.n, np.int64)
    kind[sel & ~big] = 1
    kind[sel_split & big] = 2
    kind[prune] = 3
    return kind


def densify(scene, accum, denom, normals, prm: DensifyParams, accum_abs=None):
    """Returns (new attribute dict, source index per output, child kind per
    output (0 original, 1 clone, 2 + c split child c)).  Output order: kept
    originals, then clone copies, then split children, each by ascending source
    index.  normals [n, split_count, 3] are the standard normal draws of the
    split children (passed in so that both implementations use the same)."""
    kind = decide(scene, accum, denom, prm, accum_abs)
    idx = np.arange(scene.n)
    kept = idx[(kind == 0) | (kind == 1)]
    clones = idx[kind == 1]
    splits = idx[kind == 2]
    src = np.concatenate([kept, clones, np.repeat(splits, prm.split_count)]).astype(np.int64)
    tag = np.concatenate([np.zeros(len(kept)), np.ones(len(clones)),
                          np.tile(2 + np.arange(prm.split_count), len(splits))]).astype(np.int64)
    out = {}
    for name in ("means", "scales", "quats", "opacities", "colors", "sh", "freqs", "weights"):
        a = getattr(scene, name)
        if a is not None:
            out[name] = np.asarray(a, np.float64)[src].copy()
    child = tag > 0
    out["freqs"][child] = prm.freq_reset
    out["weights"][child] = prm.weight_reset
    # split children: mean + R(q) (s * z), scale * shrink
    first_split = len(kept) + len(clones)
    for j in range(len(splits)):
        i = splits[j]
        R = quat_rot(scene.quats[i])
        s = np.asarray(scene.scales[i], np.float64)
        for c in range(prm.split_count):
            o = first_split + j * prm.split_count + c
            z = np.asarray(normals[i, c], np.float64)
            out["means"][o] = np.asarray(scene.means[i], np.float64) + R @ (s * z)
            out["scales"][o] = s * prm.split_shrink
    return out, src, tag


def periodic_reset(scene, weight_value=0.01, opacity_cap=0.02):
    """Every frequency weight := weight_value; opacity := min(opacity, cap)."""
    w = np.full_like(np.asarray(scene.weights, np.float64), weight_value)
    o = np.minimum(np.asarray(scene.opacities, np.float64), opacity_cap)
    return w, o
