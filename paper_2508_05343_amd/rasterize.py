"""Torch-facing layer over the C ABI: device scenes, per-batch buffers, the
forward/backward/loss calls and a torch.autograd.Function.

Torch provides device memory and the stream; every step of the rasterizer
runs in the HIP kernels of libgabsplat.so.  Scene attributes are kept in the
library's layouts (planar [A][n] for the geometry, frequencies and weights,
one row per primitive [n][A] for the colour coefficients) so no per-call
transposes are needed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib

TILE = 16


# ----------------------------------------------------------------- scenes
class DeviceScene:
    """Activated primitive attributes as fp32 device tensors: planar means
    [3,n], scales [3,n], quats [4,n], opacities [n], freqs [3K,n], weights
    [K,n], and per-primitive colour rows sh [n,D*3] ((d*3 + c) within a row)
    or colors [n,3]. 

    Options: attenuation (keep the z-integration factor of every cosine term),
    mip2d (Mip-Splatting's 2D filter instead of the 0.3 px^2 dilation) and
    filter3d ([n] variances of Mip-Splatting's 3D filter, e.g. from
    compute_filter3d; None = no 3D filter)."""

    def __init__(self, means, scales, quats, opacities, freqs, weights, sh=None, colors=None, sh_degree=-1,
                 attenuation=False, mip2d=False, filter3d=None):
        self.attenuation = bool(attenuation)
        self.mip2d = bool(mip2d)
        self.filter3d = filter3d
        self.means, self.scales, self.quats, self.opacities = means, scales, quats, opacities
        self.freqs, self.weights, self.sh, self.colors = freqs, weights, sh, colors
        self.sh_degree = sh_degree if sh is not None else -1
        self.n = int(means.shape[1])
        self.k = int(weights.shape[0])
        # colour coefficients are one row per primitive
        if sh is not None and tuple(sh.shape) != (self.n, 3 * (self.sh_degree + 1) ** 2):
            raise ValueError(f"sh must be [n, {3 * (self.sh_degree + 1) ** 2}] (one row per primitive), "
                             f"got {tuple(sh.shape)}")
        if colors is not None and tuple(colors.shape) != (self.n, 3):
            raise ValueError(f"colors must be [n, 3] (one row per primitive), got {tuple(colors.shape)}")

    @staticmethod
    def from_host(scene, device="cuda", attenuation=False, mip2d=False) -> "DeviceScene":
        """From AoS numpy arrays (synthetic generator layout)."""
        def planar(a):
            a = np.asarray(a, np.float32)
            return torch.from_numpy(np.ascontiguousarray(a.reshape(a.shape[0], -1).T)).to(device)

        def rows(a):
            a = np.asarray(a, np.float32)
            return torch.from_numpy(np.ascontiguousarray(a.reshape(a.shape[0], -1))).to(device)
        n = scene.means.shape[0]
        return DeviceScene(planar(scene.means), planar(scene.scales), planar(scene.quats),
                           torch.from_numpy(np.ascontiguousarray(scene.opacities, np.float32)).to(device),
                           planar(scene.freqs.reshape(n, -1)), planar(scene.weights),
                           sh=None if scene.sh is None else rows(scene.sh),
                           colors=None if scene.colors is None else rows(scene.colors),
                           sh_degree=scene.sh_degree if scene.sh is not None else -1, attenuation=attenuation,
                           mip2d=mip2d)

    def tensors(self):
        return [self.means, self.scales, self.quats, self.opacities, self.sh if self.sh is not None else self.colors,
                self.freqs, self.weights]

    def flags(self) -> int:
        f = _lib.FLAG_ATTENUATION if self.attenuation else 0
        f |= _lib.FLAG_MIP_2D if self.mip2d else 0
        f |= _lib.FLAG_MIP_3D if self.filter3d is not None else 0
        return f

    def compute_filter3d(self, cams, s: float = 0.2, margin: float = 0.15, stream=None) -> torch.Tensor:
        """Variances of Mip-Splatting's 3D filter from the training cameras
        (gabsplat_mip_filter3d), kept in self.filter3d (the same tensor across
        calls while n is unchanged, so plans built earlier stay valid)."""
        if self.filter3d is None or self.filter3d.numel() != self.n:
            self.filter3d = torch.empty(max(self.n, 1), dtype=torch.float32, device=self.means.device)
        cc = [camera_struct(c) for c in cams]
        wsb = _lib.gabsplat_mip_filter3d_workspace_size(self.n, len(cc))
        ws = torch.empty((wsb + 3) // 4, dtype=torch.int32, device=self.means.device)
        _lib.gabsplat_mip_filter3d(self.means, self.n, cc, s, margin, self.filter3d, ws, stream)
        return self.filter3d

    def cstruct(self) -> _lib.Scene:
        s = _lib.Scene()
        s.n, s.k, s.sh_degree = self.n, self.k, max(self.sh_degree, 0)
        s.flags = self.flags()
        s.filter3d = _lib.ptr(self.filter3d)
        s.means, s.scales, s.quats = _lib.ptr(self.means), _lib.ptr(self.scales), _lib.ptr(self.quats)
        s.opacities = _lib.ptr(self.opacities)
        s.sh = _lib.ptr(self.sh) if self.sh is not None else None
        s.colors = _lib.ptr(self.colors) if self.colors is not None else None
        s.freqs, s.weights = _lib.ptr(self.freqs), _lib.ptr(self.weights)
        return s

    def nbytes(self) -> int:
        return sum(t.numel() * 4 for t in self.tensors() if t is not None)


def camera_struct(cam) -> _lib.Camera:
    c = _lib.Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    R = np.asarray(cam.R, np.float32)
    t = np.asarray(cam.t, np.float32)
    w2c = np.concatenate([R, t[:, None]], 1).reshape(-1)
    for i in range(12):
        c.world_to_cam[i] = float(w2c[i])
    for i in range(3):
        c.cam_pos[i] = float(cam.eye[i])
        c.bg[i] = float(cam.bg[i])
    c.near_plane = float(cam.near)
    return c


# ------------------------------------------------------------------ plans
@dataclass
class ViewLayout:
    width: int
    height: int
    tile_offset: int
    pixel_offset: int
    item_offset: int


class RenderPlan:
    """Buffers and calls for one batch of views over one or more scenes.

    Allocations happen here (and on capacity growth), never inside the
    per-step calls."""

    def __init__(self, scenes: Sequence[DeviceScene], cams: Sequence, scene_of_view: Optional[Sequence[int]] = None,
                 pair_capacity: Optional[int] = None, device="cuda", want_keys=False, abs_mean2d=False):
        self.scenes = list(scenes)
        # backward flags: abs_mean2d adds the AbsGS per-pixel absolute mean gradients to grad2d
        self.grad_flags = _lib.GRAD_ABS_MEAN2D if abs_mean2d else 0
        self.cams = list(cams)
        self.scene_of_view = None if scene_of_view is None else [int(s) for s in scene_of_view]
        sv = self.scene_of_view or [0] * len(self.cams)
        self.k = self.scenes[0].k
        self.device = device
        self.c_scenes = [s.cstruct() for s in self.scenes]
        self.c_cams = [camera_struct(c) for c in self.cams]
        self.layout: List[ViewLayout] = []
        items = pix = tiles = 0
        for c, s in zip(self.cams, sv):
            self.layout.append(ViewLayout(c.width, c.height, tiles, pix, items))
            items += self.scenes[s].n
            pix += c.width * c.height
            tiles += ((c.width + TILE - 1) // TILE) * ((c.height + TILE - 1) // TILE)
        self.items, self.pixels, self.tiles = items, pix, tiles
        rf = _lib.gabsplat_record_floats(self.k)
        self.rec = torch.empty((max(items, 1), rf), dtype=torch.float32, device=device)
        self.depth = torch.empty(max(items, 1), dtype=torch.float32, device=device)
        self.rect = torch.empty((max(items, 1), 2), dtype=torch.int32, device=device)
        self.tiles_touched = torch.empty(max(items, 1), dtype=torch.int32, device=device)
        vb = _lib.gabsplat_views_bytes(len(self.cams), len(self.scenes))
        self.views = torch.empty((vb + 15) // 16 * 4, dtype=torch.int32, device=device)
        self.geom = _lib.Geom()
        self.geom.k = self.k
        self.geom.rec, self.geom.depth = _lib.ptr(self.rec), _lib.ptr(self.depth)
        self.geom.rect, self.geom.tiles = _lib.ptr(self.rect), _lib.ptr(self.tiles_touched)
        self.geom.views = _lib.ptr(self.views)
        self.ranges = torch.empty((max(tiles, 1), 2), dtype=torch.int32, device=device)
        self.num_pairs = torch.zeros(1, dtype=torch.int64, device=device)
        self.overflow = torch.zeros(1, dtype=torch.int32, device=device)
        self.image = torch.empty(max(3 * pix, 1), dtype=torch.float32, device=device)
        self.final_T = torch.empty(max(pix, 1), dtype=torch.float32, device=device)
        self.n_contrib = torch.empty(max(pix, 1), dtype=torch.int32, device=device)
        self.want_keys = want_keys
        self.capacity = 0
        self._alloc_pairs(pair_capacity if pair_capacity is not None else max(1 << 16, 8 * items))
        self.grad2d = None

    def _alloc_pairs(self, cap: int):
        cap = int(cap)
        self.capacity = cap
        self.vals = torch.empty(max(cap, 1), dtype=torch.int32, device=self.device)
        self.keys = torch.empty(max(cap, 1), dtype=torch.int64, device=self.device) if self.want_keys else None
        wsb = _lib.gabsplat_bin_sort_workspace_size(self.items, cap, self.tiles)
        self.ws = torch.empty((wsb + 255) // 256 * 64, dtype=torch.int32, device=self.device)

    # ----- stages
    def preprocess(self, stream=None):
        _lib.gabsplat_preprocess(self.c_scenes, self.scene_of_view, self.c_cams, self.geom, stream)

    def bin_sort(self, stream=None):
        _lib.gabsplat_bin_sort(self.geom, self.c_cams, self.items, self.ws, self.keys, self.vals, self.capacity,
                               self.ranges, self.num_pairs, self.overflow, stream)

    def render_fwd(self, stream=None, eval_counts=None, freq_map=None):
        _lib.gabsplat_render_fwd(self.geom, self.vals, self.ranges, self.c_cams, self.image, self.final_T,
                                 self.n_contrib, self.overflow, stream, eval_counts=eval_counts, freq_map=freq_map)

    def forward(self, check_overflow=True, stream=None):
        """preprocess -> bin_sort -> render_fwd.  With check_overflow the pair
        count is read back (a host sync) and the bin sort retried with a
        larger capacity if it overflowed."""
        self.preprocess(stream)
        self.bin_sort(stream)
        if check_overflow and _lib.gabsplat_read_overflow(self.overflow, stream):
            need = int(self.num_pairs.item())
            self._alloc_pairs(int(need * 1.25) + 1024)
            self.bin_sort(stream)
            if _lib.gabsplat_read_overflow(self.overflow, stream):
                raise _lib.GabsplatError(_lib.CAPACITY_EXCEEDED, "pair capacity still exceeded after growth")
        self.render_fwd(stream)
        return self.image

    def backward(self, dl_dimage, grads: Sequence[dict], stream=None, accumulate=True):
        """dl_dimage has the layout of self.image; grads[s] maps attribute name
        -> tensor (same layout as the scene) that receives the gradient, added
        to it (accumulate=True) or overwriting it."""
        if self.grad2d is None:
            gf = _lib.gabsplat_grad2d_stride(self.k, self.grad_flags)
            self.grad2d = torch.empty((max(self.items, 1), gf), dtype=torch.float32, device=self.device)
        gs = []
        for g in grads:
            c = _lib.SceneGrads()
            c.accumulate = 1 if accumulate else 0
            c.flags = self.grad_flags
            for name in ("means", "scales", "quats", "opacities", "sh", "colors", "freqs", "weights"):
                setattr(c, name, _lib.ptr(g.get(name)))
            c.grad2d = _lib.ptr(self.grad2d)
            gs.append(c)
        _lib.gabsplat_render_bwd(self.c_scenes, self.scene_of_view, self.c_cams, self.geom, self.vals, self.ranges,
                                 self.final_T, self.n_contrib, dl_dimage, gs, self.overflow, stream)

    # ----- views of the outputs
    def view_image(self, v: int) -> torch.Tensor:
        L = self.layout[v]
        hw = L.width * L.height
        return self.image[3 * L.pixel_offset:3 * (L.pixel_offset + hw)].view(3, L.height, L.width)

    def view_final_T(self, v: int) -> torch.Tensor:
        L = self.layout[v]
        return self.final_T[L.pixel_offset:L.pixel_offset + L.width * L.height].view(L.height, L.width)

    def view_n_contrib(self, v: int) -> torch.Tensor:
        L = self.layout[v]
        return self.n_contrib[L.pixel_offset:L.pixel_offset + L.width * L.height].view(L.height, L.width)

    def view_ranges(self, v: int) -> torch.Tensor:
        L = self.layout[v]
        c = self.cams[v]
        nt = ((c.width + TILE - 1) // TILE) * ((c.height + TILE - 1) // TILE)
        return self.ranges[L.tile_offset:L.tile_offset + nt]

    def record_fields(self):
        """Named views of the render records (testing and inspection)."""
        r = self.rec[:self.items]
        k = self.k
        log2e = 1.0 / math.log(2.0)
        out = dict(mu2d=r[:, 0:2], conic=torch.stack([r[:, 2] / (-0.5 * log2e), r[:, 3] / (-log2e),
                                                      r[:, 4] / (-0.5 * log2e)], 1),
                   opacity=torch.exp2(r[:, 5]), rgb=r[:, 6:9], w0=r[:, 9])
        if k:
            f = r[:, 10:10 + 3 * k].reshape(-1, k, 3)
            out["f2d"] = f[:, :, 0:2]
            out["w"] = f[:, :, 2]
        return out


class LossBuffers:
    def __init__(self, c, h, w, device="cuda"):
        self.ws = torch.empty((_lib.gabsplat_loss_workspace_size(c, h, w) + 3) // 4, dtype=torch.float32,
                              device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.grad = torch.empty((c, h, w), dtype=torch.float32, device=device)

    def __call__(self, x, y, lam=0.2, stream=None):
        _lib.gabsplat_loss_l1_dssim(x, y, lam, self.loss, self.grad, self.ws, stream)
        return self.loss, self.grad


# --------------------------------------------------------------- autograd
class GaborRasterize(torch.autograd.Function):
    """image = rasterize(means, scales, quats, opacities, color, freqs, weights)
    for one scene and a list of cameras; `color` is the SH tensor [n, D*3]
    (sh_degree >= 0) or RGB [n, 3].  Returns the flat image buffer of the plan
    (views back to back, [3][H][W] each)."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, color, freqs, weights, plan: RenderPlan):
        img = plan.forward(check_overflow=True)
        ctx.plan = plan
        return img.clone()

    @staticmethod
    def backward(ctx, dl_dimage):
        plan: RenderPlan = ctx.plan
        sc = plan.scenes[0]
        g = {name: torch.zeros_like(getattr(sc, name)) for name in
             ("means", "scales", "quats", "opacities", "freqs", "weights")}
        if sc.sh is not None:
            g["sh"] = torch.zeros_like(sc.sh)
        else:
            g["colors"] = torch.zeros_like(sc.colors)
        plan.backward(dl_dimage.contiguous(), [g])
        col = g.get("sh", g.get("colors"))
        return g["means"], g["scales"], g["quats"], g["opacities"], col, g["freqs"], g["weights"], None


def rasterize(scene: DeviceScene, plan: RenderPlan):
    """Differentiable render of `plan`'s views of `scene` (flat image buffer)."""
    col = scene.sh if scene.sh is not None else scene.colors
    return GaborRasterize.apply(scene.means, scene.scales, scene.quats, scene.opacities, col, scene.freqs,
                                scene.weights, plan)
