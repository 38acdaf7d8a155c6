"""Torch-facing layer over the C ABI: device scenes, per-batch buffers, the
forward/backward/loss calls and a torch.autograd.Function.

Torch provides device memory and the stream; every step of the rasterizer
runs in the HIP kernels of libgabsplat.so.  Scene attributes are kept in the
library's layouts (planar [A][n] for the geometry, frequencies and weights,
one row per primitive [n][A] for the colour coefficients) so no per-call
transposes are needed.
"""
from __future__ import annotations

import copy
import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib

TILE = 16


# ----------------------------------------------------------------- scenes
def check_device_tensor(name: str, t, shape, device=None, check_device: bool = True):
    """Raises ValueError unless ``t`` is a contiguous float32 device tensor of
    exactly ``shape`` (on ``device`` when given); returns its device.  The
    kernels read these buffers through raw pointers with the layouts of the C
    ABI, so a transposed view, a short array or a host tensor would be misread
    or read out of bounds.  Checked in the order dtype, shape, layout, device."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor, got {type(t).__name__}")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (the library reads it through a raw pointer)")
    if not check_device:
        return t.device
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor, got device {t.device}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the other attributes on {device}")
    return t.device


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
        if (sh is None) == (colors is None):
            raise ValueError("exactly one of sh and colors must be given")
        if sh is not None and not 0 <= int(sh_degree) <= 3:
            raise ValueError(f"sh_degree must be in [0, 3] with sh, got {sh_degree}")
        if not isinstance(weights, torch.Tensor) or weights.dim() != 2:
            raise ValueError("weights must be a [K, n] tensor")
        if not isinstance(means, torch.Tensor) or means.dim() != 2:
            raise ValueError("means must be a [3, n] tensor")
        self.n = int(means.shape[1])
        self.k = int(weights.shape[0])
        if not 0 <= self.k <= 8:
            raise ValueError(f"K = {self.k} frequency components: at most 8 are supported")
        self.sh_degree = int(sh_degree) if sh is not None else -1
        n, k = self.n, self.k
        shapes = dict(means=(3, n), scales=(3, n), quats=(4, n), opacities=(n,), freqs=(3 * k, n), weights=(k, n))
        # colour coefficients are one row per primitive
        if sh is not None:
            shapes["sh"] = (n, 3 * (self.sh_degree + 1) ** 2)
        else:
            shapes["colors"] = (n, 3)
        if filter3d is not None:
            shapes["filter3d"] = (n,)
        given = dict(means=means, scales=scales, quats=quats, opacities=opacities, freqs=freqs, weights=weights,
                     sh=sh, colors=colors, filter3d=filter3d)
        # layouts of every attribute first, then where they live
        for name, shape in shapes.items():
            check_device_tensor(name, given[name], shape, check_device=False)
        dev = None
        for name, shape in shapes.items():
            dev = check_device_tensor(name, given[name], shape, dev)
        self.means, self.scales, self.quats, self.opacities = means, scales, quats, opacities
        self.freqs, self.weights, self.sh, self.colors = freqs, weights, sh, colors
        self.filter3d = filter3d
        self.rows = None  # row-major quats/freqs/weights (with_rows), read by the projection when set

    def with_rows(self, stream=None) -> "DeviceScene":
        """The same scene (the same tensors) plus a row-major copy of every
        primitive's quaternion, frequencies and weights (gabsplat_pack_rows,
        one 128-byte line per primitive for K <= 7), which the projection
        reads instead of their planes: the planes' lines hold mostly culled
        neighbours of each visible primitive.  For scenes that stay fixed
        (serving): the copy is not updated when the planes change."""
        ds = copy.copy(self)
        rs = _lib.gabsplat_row_floats(self.k)
        ds.rows = torch.empty((max(self.n, 1), rs), dtype=torch.float32, device=self.means.device)
        _lib.gabsplat_pack_rows(self.cstruct(), ds.rows, stream)
        return ds

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
        s.rows = _lib.ptr(self.rows) if self.rows is not None else None
        return s

    def nbytes(self) -> int:
        rows = self.rows.numel() * 4 if self.rows is not None else 0
        return sum(t.numel() * 4 for t in self.tensors() if t is not None) + rows


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
_ITEMSIZE = {torch.float32: 4, torch.int32: 4, torch.int64: 8}


def plan_buffer_specs(k: int, items: int, pixels: int, tiles: int, n_views: int, n_scenes: int, capacity: int,
                      want_keys: bool = False) -> Dict[str, tuple]:
    """The device buffers a RenderPlan allocates for its forward: name ->
    (shape, dtype).  The plan allocates exactly these, so their sum is the
    plan's device footprint (serving admits batches by it)."""
    rf = _lib.gabsplat_record_floats(k)
    vb = _lib.gabsplat_views_bytes(n_views, n_scenes)
    it, px, tl, cap = max(items, 1), max(pixels, 1), max(tiles, 1), max(int(capacity), 1)
    wsb = _lib.gabsplat_bin_sort_workspace_size(items, int(capacity), tiles)
    f32, i32, i64 = torch.float32, torch.int32, torch.int64
    specs = dict(rec=((it, rf), f32), depth=((it,), f32), rect=((it, 2), i32), tiles_touched=((it,), i32),
                 views=(((vb + 15) // 16 * 4,), i32), ranges_buf=((3 * tl,), i32), num_pairs=((1,), i64),
                 overflow=((1,), i32), image=((3 * px,), f32), final_T=((px,), f32), n_contrib=((px,), i32),
                 vals=((cap,), i32), ws=(((wsb + 255) // 256 * 64,), i32))
    if want_keys:
        specs["keys"] = ((cap,), i64)
    return specs


def specs_nbytes(specs: Dict[str, tuple]) -> int:
    return sum(math.prod(shape) * _ITEMSIZE[dt] for shape, dt in specs.values())


def block_bytes(nbytes: int) -> int:
    """Upper bound of the device bytes torch's caching allocator charges for
    one buffer of `nbytes`: requests round up to 512 bytes, and one above
    1 MiB served from a larger cached block keeps up to 1 MiB of that block
    unsplit."""
    r = (max(int(nbytes), 1) + 511) // 512 * 512
    return r + ((1 << 20) if r > (1 << 20) else 0)


def specs_block_bytes(specs: Dict[str, tuple]) -> int:
    """Allocator-charged bytes (block_bytes) of a set of buffer specs."""
    return sum(block_bytes(math.prod(shape) * _ITEMSIZE[dt]) for shape, dt in specs.values())


class DeviceArena:
    """Grow-only device buffers that successive plans reuse (serving keeps one
    per stream): a plan takes each of its buffers as a view of the arena's
    buffer of the same name, which is reallocated only when it is too small.
    A plan built on an arena must be done with (its results copied out)
    before the next plan takes the same arena."""

    def __init__(self, device="cuda"):
        self.device = device
        self.bufs: Dict[str, torch.Tensor] = {}
        self.views: Dict[str, tuple] = {}  # name -> (shape, view) last handed out
        self.allocations = 0  # buffers allocated (first use or growth) so far

    def take(self, name: str, shape: tuple, dtype) -> torch.Tensor:
        shape = tuple(shape)
        numel = math.prod(shape)
        b = self.bufs.get(name)
        if b is None or b.dtype != dtype or b.numel() < numel:
            # the old buffer (and the view of it) is dropped, its last
            # reference included, before the new one is allocated: the two
            # are never held together
            b = None
            self.views.pop(name, None)
            self.bufs.pop(name, None)
            b = torch.empty(numel, dtype=dtype, device=self.device)
            self.bufs[name] = b
            self.allocations += 1
        v = self.views.get(name)
        if v is not None and v[0] == shape:
            return v[1]  # the same view again (no per-batch view construction)
        view = b[:numel].view(shape)
        self.views[name] = (shape, view)
        return view

    def nbytes(self) -> int:
        """Allocator-charged bytes (block_bytes) of the buffers held."""
        return sum(block_bytes(b.numel() * b.element_size()) for b in self.bufs.values())

    def nbytes_after(self, specs: Dict[str, tuple]) -> int:
        """Allocator-charged bytes held once a plan with these buffer specs
        has taken its buffers."""
        held = {n: b.numel() * b.element_size() for n, b in self.bufs.items()}
        for n, (shape, dt) in specs.items():
            held[n] = max(held.get(n, 0), math.prod(shape) * _ITEMSIZE[dt])
        return sum(block_bytes(v) for v in held.values())

    def release(self):
        self.views.clear()
        self.bufs.clear()


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
                 pair_capacity: Optional[int] = None, device="cuda", want_keys=False, abs_mean2d=False,
                 arena: Optional[DeviceArena] = None):
        self.arena = arena
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
        self.want_keys = want_keys
        self.capacity = int(pair_capacity if pair_capacity is not None else max(1 << 16, 8 * items))
        specs = plan_buffer_specs(self.k, items, pix, tiles, len(self.cams), len(self.scenes), self.capacity,
                                  want_keys)
        allocated = arena.allocations if arena is not None else None
        for name, (shape, dt) in specs.items():
            setattr(self, name, self._take(name, shape, dt))
        # [tiles][2] ranges, then the blend's dispatch order of the tiles
        self.ranges = self.ranges_buf[:2 * max(tiles, 1)].view(max(tiles, 1), 2)
        # defined before the first bin sort (which rewrites both); buffers an
        # arena hands out again already hold a bin sort's values
        if arena is None or arena.allocations != allocated:
            self.num_pairs.zero_()
            self.overflow.zero_()
        if not want_keys:
            self.keys = None
        self.geom = _lib.Geom()
        self.geom.k = self.k
        self.geom.rec, self.geom.depth = _lib.ptr(self.rec), _lib.ptr(self.depth)
        self.geom.rect, self.geom.tiles = _lib.ptr(self.rect), _lib.ptr(self.tiles_touched)
        self.geom.views = _lib.ptr(self.views)
        self.grad2d = None
        # bumped by every stage that rewrites the buffers a backward reads
        # (records, pair lists, final_T, n_contrib); an autograd graph keeps
        # the value of its forward and refuses a backward after a newer run
        self.generation = 0

    def bind_scene(self, index: int, scene: DeviceScene):
        """Renders ``scene`` in place of scene ``index`` from now on.  It must
        have the same primitive count, component count, colour mode and
        options (the plan's buffers are sized and laid out for them)."""
        old = self.scenes[index]
        if (scene.n, scene.k, scene.sh_degree, scene.flags()) != (old.n, old.k, old.sh_degree, old.flags()) or \
                (scene.sh is None) != (old.sh is None):
            raise ValueError(f"scene {index}: (n, k, sh_degree, flags) = {(scene.n, scene.k, scene.sh_degree, scene.flags())}"
                             f" does not match the plan's {(old.n, old.k, old.sh_degree, old.flags())}")
        if scene.means.device != torch.device(self.device) and str(self.device) != "cuda":
            raise ValueError(f"scene on {scene.means.device}, plan on {self.device}")
        self.scenes[index] = scene
        self.c_scenes[index] = scene.cstruct()

    def _take(self, name: str, shape: tuple, dtype) -> torch.Tensor:
        if self.arena is not None:
            return self.arena.take(name, shape, dtype)
        return torch.empty(shape, dtype=dtype, device=self.device)

    def buffer_specs(self, capacity: Optional[int] = None) -> Dict[str, tuple]:
        """This plan's buffer specs (plan_buffer_specs), at another pair
        capacity if given."""
        return plan_buffer_specs(self.k, self.items, self.pixels, self.tiles, len(self.cams), len(self.scenes),
                                 self.capacity if capacity is None else capacity, self.want_keys)

    def _alloc_pairs(self, cap: int):
        cap = int(cap)
        self.capacity = cap
        specs = self.buffer_specs(cap)
        for name in ("vals", "keys", "ws"):
            if name in specs:
                setattr(self, name, None)  # the old buffer is freed before the larger one is taken
                setattr(self, name, self._take(name, *specs[name]))

    # ----- stages
    def preprocess(self, stream=None):
        self.generation += 1
        _lib.gabsplat_preprocess(self.c_scenes, self.scene_of_view, self.c_cams, self.geom, stream)

    def bin_sort(self, stream=None):
        self.generation += 1
        _lib.gabsplat_bin_sort(self.geom, self.c_cams, self.items, self.ws, self.keys, self.vals, self.capacity,
                               self.ranges_buf, self.num_pairs, self.overflow, stream)

    def render_fwd(self, stream=None, eval_counts=None, freq_map=None):
        self.generation += 1
        _lib.gabsplat_render_fwd(self.geom, self.vals, self.ranges_buf, self.c_cams, self.image, self.final_T,
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

    def backward(self, dl_dimage, grads: Sequence[dict], stream=None, accumulate=True, stages=None):
        """dl_dimage has the layout of self.image; grads[s] maps attribute name
        -> tensor (same layout as the scene) that receives the gradient, added
        to it (accumulate=True) or overwriting it.  stages (default both):
        _lib.BWD_BLEND (the image-plane gradients into grad2d) and/or
        _lib.BWD_PROJECT (grad2d through the projection into grads), to run
        the two parts as separate calls."""
        if not isinstance(dl_dimage, torch.Tensor) or dl_dimage.numel() != 3 * self.pixels:
            raise ValueError(f"dl_dimage must hold the plan's {3 * self.pixels} image values")
        check_device_tensor("dl_dimage", dl_dimage, tuple(dl_dimage.shape), self.image.device)
        if len(grads) != len(self.scenes):
            raise ValueError(f"{len(grads)} gradient sets for {len(self.scenes)} scenes")
        if self.grad2d is None:
            gf = _lib.gabsplat_grad2d_stride(self.k, self.grad_flags)
            self.grad2d = torch.empty((max(self.items, 1), gf), dtype=torch.float32, device=self.device)
        gs = []
        for sc, g in zip(self.scenes, grads):
            c = _lib.SceneGrads()
            c.accumulate = 1 if accumulate else 0
            c.flags = self.grad_flags
            for name in ("means", "scales", "quats", "opacities", "sh", "colors", "freqs", "weights"):
                t = g.get(name)
                if t is not None:
                    ref = getattr(sc, name)
                    if ref is None:
                        raise ValueError(f"gradient for {name}, which the scene does not have")
                    check_device_tensor(f"grads[{name}]", t, tuple(ref.shape), ref.device)
                setattr(c, name, _lib.ptr(t))
            c.grad2d = _lib.ptr(self.grad2d)
            gs.append(c)
        if stages is None:
            _lib.gabsplat_render_bwd(self.c_scenes, self.scene_of_view, self.c_cams, self.geom, self.vals,
                                     self.ranges_buf, self.final_T, self.n_contrib, dl_dimage, gs, self.overflow, stream)
        else:
            _lib.gabsplat_render_bwd_stages(self.c_scenes, self.scene_of_view, self.c_cams, self.geom, self.vals,
                                            self.ranges_buf, self.final_T, self.n_contrib, dl_dimage, gs,
                                            self.overflow, stages, stream)

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
        lo = 10 + 3 * k  # residuals of the mean's float32 rounding
        out = dict(mu2d=r[:, 0:2].double() + r[:, lo:lo + 2].double(), conic=torch.stack([r[:, 2] / (-0.5 * log2e), r[:, 3] / (-log2e),
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
    """image = GaborRasterize.apply(means, scales, quats, opacities, color,
    freqs, weights, plan): the activated attributes of one scene (the layouts
    of DeviceScene; ``color`` is the SH rows [n, 3 (deg+1)^2] or the RGB rows
    [n, 3], as the plan's scene) rendered through every camera of ``plan``.
    Returns the flat image (views back to back, [3][H][W] each).

    The tensors given are the ones rendered: they are validated and bound to
    the plan as its scene for this call, so they may be the outputs of torch
    ops (exp of log-scales, sigmoid of logits, Sec. 3.4.1).  The backward
    reads the plan's per-call buffers, so a plan carries one live graph at a
    time: a backward after the plan has run again raises."""

    @staticmethod
    def forward(ctx, means, scales, quats, opacities, color, freqs, weights, plan: RenderPlan):
        if len(plan.scenes) != 1:
            raise ValueError("GaborRasterize renders one scene; the plan has several")
        tmpl = plan.scenes[0]
        has_sh = tmpl.sh is not None
        ds = DeviceScene(means, scales, quats, opacities, freqs, weights, sh=color if has_sh else None,
                         colors=None if has_sh else color, sh_degree=tmpl.sh_degree, attenuation=tmpl.attenuation,
                         mip2d=tmpl.mip2d, filter3d=tmpl.filter3d)
        plan.bind_scene(0, ds)
        img = plan.forward(check_overflow=True)
        ctx.plan, ctx.scene, ctx.generation = plan, ds, plan.generation
        return img.clone()

    @staticmethod
    def backward(ctx, dl_dimage):
        plan: RenderPlan = ctx.plan
        if plan.generation != ctx.generation or plan.scenes[0] is not ctx.scene:
            raise RuntimeError("GaborRasterize: the plan has run again since this forward; its buffers no longer "
                               "hold this graph's state (use one plan per live graph)")
        sc = ctx.scene
        names = ("means", "scales", "quats", "opacities", "color", "freqs", "weights")
        g = {}
        for i, name in enumerate(names):
            if not ctx.needs_input_grad[i]:
                continue
            attr = ("sh" if sc.sh is not None else "colors") if name == "color" else name
            g[attr] = torch.empty_like(getattr(sc, attr))
        if g:
            plan.backward(dl_dimage.contiguous().view(-1), [g], accumulate=False)
        col = g.get("sh", g.get("colors"))
        return (g.get("means"), g.get("scales"), g.get("quats"), g.get("opacities"), col, g.get("freqs"),
                g.get("weights"), None)


def rasterize(plan: RenderPlan, means, scales, quats, opacities, color, freqs, weights):
    """Differentiable render of the given activated attributes through the
    plan's cameras (flat image buffer); see GaborRasterize."""
    return GaborRasterize.apply(means, scales, quats, opacities, color, freqs, weights, plan)


def rasterize_scene(scene: DeviceScene, plan: RenderPlan):
    """rasterize() of a DeviceScene's tensors."""
    col = scene.sh if scene.sh is not None else scene.colors
    return rasterize(plan, scene.means, scene.scales, scene.quats, scene.opacities, col, scene.freqs, scene.weights)


class PhotometricLoss(torch.autograd.Function):
    """L = (1 - lam) mean|x - y| + lam (1 - mean SSIM(x, y)) of Sec. 3.4.1
    through the library's loss kernels; x, y [C, H, W] float32 device tensors.
    The gradient with respect to x is computed by the forward call (one kernel
    pass yields both) and scaled by the incoming gradient."""

    @staticmethod
    def forward(ctx, x, y, lam, buffers):
        c, h, w = x.shape
        check_device_tensor("x", x, (c, h, w))
        check_device_tensor("y", y, (c, h, w), x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        grad = torch.empty_like(x)
        if buffers is None:
            buffers = LossBuffers(c, h, w, device=x.device)
        _lib.gabsplat_loss_l1_dssim(x, y, float(lam), loss, grad, buffers.ws, None)
        ctx.save_for_backward(grad)
        return loss[0]

    @staticmethod
    def backward(ctx, go):
        (grad,) = ctx.saved_tensors
        return grad * go, None, None, None


def photometric_loss(x, y, lam: float = 0.2, buffers: Optional["LossBuffers"] = None):
    """Differentiable L1 + lam D-SSIM loss (the training objective of Sec. 3.4.1)."""
    return PhotometricLoss.apply(x, y, lam, buffers)
