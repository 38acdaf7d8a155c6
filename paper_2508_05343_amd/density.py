"""Frequency-adaptive density control on device scenes (torch for memory,
the HIP kernels of libgabsplat.so for the work)."""
from __future__ import annotations

from typing import Optional, Tuple

import torch

from . import _lib
from .rasterize import DeviceScene, RenderPlan

# attributes stored one row per primitive ([n][A]); the others are planar [A][n]
ROWS = ("sh", "colors")


def default_params(scene_extent: float = 1.0, **kw) -> _lib.DensifyParams:
    p = _lib.DensifyParams()
    p.grad_threshold, p.percent_dense, p.scene_extent = 0.0002, 0.01, float(scene_extent)
    p.min_opacity, p.max_world_frac, p.prune_big = 0.01, 0.1, 0
    p.freq_reset, p.weight_reset, p.split_shrink, p.split_count = 0.001, 0.01, 1.0 / 1.6, 2
    p.abs_grad_threshold = 0.0
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def scene_out_struct(ds: DeviceScene) -> _lib.SceneOut:
    o = _lib.SceneOut()
    o.n, o.k, o.sh_degree = ds.n, ds.k, max(ds.sh_degree, 0)
    o.flags = _lib.FLAG_ATTENUATION if ds.attenuation else 0
    for name in ("means", "scales", "quats", "opacities", "sh", "colors", "freqs", "weights"):
        setattr(o, name, _lib.ptr(getattr(ds, name)))
    return o


class DensityStats:
    """Per-primitive accumulated view-space gradient norm and visible count;
    with abs_stat also the AbsGS homodirectional statistic (the plans fed to
    accumulate() must then be built with abs_mean2d=True)."""

    def __init__(self, n: int, device="cuda", abs_stat=False):
        self.accum = torch.zeros(n, dtype=torch.float32, device=device)
        self.denom = torch.zeros(n, dtype=torch.float32, device=device)
        self.accum_abs = torch.zeros(n, dtype=torch.float32, device=device) if abs_stat else None

    def accumulate(self, plan: RenderPlan, stream=None):
        """After plan.backward(): add this batch's views (single-scene plan)."""
        if plan.grad2d is None:
            raise RuntimeError("accumulate() needs the image-plane gradients of a backward pass")
        if (self.accum_abs is not None) != bool(plan.grad_flags & _lib.GRAD_ABS_MEAN2D):
            raise ValueError("the absolute statistic needs a plan built with abs_mean2d=True (and only then)")
        _lib.gabsplat_densify_stats(plan.geom, plan.c_cams, plan.scenes[0].n, plan.grad2d, plan.grad_flags,
                                    self.accum, self.accum_abs, self.denom, stream)


def densify(ds: DeviceScene, stats: DensityStats, normals: torch.Tensor, params: _lib.DensifyParams,
            stream=None) -> Tuple[DeviceScene, torch.Tensor, torch.Tensor]:
    """Returns the new scene and, per new primitive, its source index and tag
    (0 kept, 1 clone copy, 2 + c split child c).  Reads the new count back
    (one host synchronisation).  The new scene keeps the attenuation and 2D
    filter options; a 3D filter must be recomputed for it
    (compute_filter3d) before it is rendered with one."""
    n, dev = ds.n, ds.means.device
    cap = n * (1 + max(1, params.split_count))
    bufs = {}
    for name in ("means", "scales", "quats", "opacities", "sh", "colors", "freqs", "weights"):
        t = getattr(ds, name)
        if t is None:
            bufs[name] = None
            continue
        per_prim = t.shape[1] if name in ROWS else (t.shape[0] if t.dim() == 2 else 1)
        bufs[name] = torch.empty(per_prim * max(cap, 1), dtype=torch.float32, device=dev)
    out = _lib.SceneOut()
    out.n, out.k, out.sh_degree = cap, ds.k, max(ds.sh_degree, 0)
    for name, b in bufs.items():
        setattr(out, name, _lib.ptr(b))
    src = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    tag = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    n_out = torch.zeros(1, dtype=torch.int64, device=dev)
    ovf = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty((_lib.gabsplat_densify_workspace_size(n) + 3) // 4, dtype=torch.int32, device=dev)
    _lib.gabsplat_densify(ds.cstruct(), stats.accum, stats.denom, stats.accum_abs, normals, params, out, cap, src, tag,
                          n_out, ovf, ws, stream)
    m = int(n_out.item())
    if int(ovf.item()):
        raise _lib.GabsplatError(_lib.CAPACITY_EXCEEDED, "densify output larger than its capacity")

    def view(name):
        b = bufs[name]
        if b is None:
            return None
        t = getattr(ds, name)
        if t.dim() == 1:
            return b[:m].clone()
        if name in ROWS:
            return b[:m * t.shape[1]].view(m, t.shape[1]).clone()
        return b[:t.shape[0] * m].view(t.shape[0], m).clone()
    new = DeviceScene(view("means"), view("scales"), view("quats"), view("opacities"), view("freqs"),
                      view("weights"), sh=view("sh"), colors=view("colors"), sh_degree=ds.sh_degree,
                      attenuation=ds.attenuation, mip2d=ds.mip2d)
    return new, src[:m].clone(), tag[:m].clone()


def reset_frequency_weights(ds: DeviceScene, weight_value: float = 0.01, opacity_cap: float = 0.02, stream=None):
    _lib.gabsplat_reset_frequency_weights(scene_out_struct(ds), weight_value, opacity_cap, stream)
