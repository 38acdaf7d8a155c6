"""ctypes binding of libgabsplat.so (argument marshalling only).

The functions below carry the names of the C entry points declared in
include/gabsplat.h.  They take torch tensors (device memory) and small host
structs, pass raw pointers and the current HIP stream, and raise GabsplatError
on a non-OK status.  There is no fallback: if the library has not been built
(``python -m paper_2508_05343_amd.build``) every call raises.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_float, c_int32, c_int64, c_size_t, c_uint32, c_void_p
from typing import Optional, Sequence

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgabsplat.so")
# the argument layouts this binding marshals (GABSPLAT_ABI_VERSION)
ABI_VERSION = 7

EXPORTS = (
    "gabsplat_abi_version", "gabsplat_status_string", "gabsplat_record_floats", "gabsplat_grad2d_floats",
    "gabsplat_views_bytes", "gabsplat_bin_sort_workspace_size", "gabsplat_check_device",
    "gabsplat_preprocess", "gabsplat_bin_sort", "gabsplat_render_fwd", "gabsplat_render_bwd",
    "gabsplat_loss_workspace_size", "gabsplat_loss_l1_dssim", "gabsplat_read_overflow",
    "gabsplat_densify_stats", "gabsplat_densify_workspace_size", "gabsplat_densify",
    "gabsplat_reset_frequency_weights", "gabsplat_grad2d_stride", "gabsplat_mip_filter3d_workspace_size",
    "gabsplat_mip_filter3d", "gabsplat_loss_l1_dssim_noalloc", "gabsplat_render_bwd_stages",
    "gabsplat_row_floats", "gabsplat_pack_rows",
)

OK, INVALID_ARGUMENT, WORKSPACE_TOO_SMALL, CAPACITY_EXCEEDED, HIP_ERROR, UNSUPPORTED_DEVICE, SCRATCH_LIMIT = range(7)
# GABSPLAT_LOSS_NOALLOC_SCRATCH_BYTES
LOSS_NOALLOC_SCRATCH_BYTES = 83886080
# GABSPLAT_BWD_BLEND, GABSPLAT_BWD_PROJECT
BWD_BLEND, BWD_PROJECT = 1, 2
FLAG_ATTENUATION = 1
FLAG_MIP_2D = 2
FLAG_MIP_3D = 4
GRAD_ABS_MEAN2D = 1


class GabsplatError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class Scene(ctypes.Structure):
    _fields_ = [("n", c_int64), ("k", c_int32), ("sh_degree", c_int32), ("flags", c_int32), ("pad", c_int32),
                ("means", c_void_p), ("scales", c_void_p), ("quats", c_void_p), ("opacities", c_void_p),
                ("sh", c_void_p), ("colors", c_void_p), ("freqs", c_void_p), ("weights", c_void_p),
                ("filter3d", c_void_p), ("rows", c_void_p)]


class Camera(ctypes.Structure):
    _fields_ = [("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("world_to_cam", c_float * 12), ("cam_pos", c_float * 3),
                ("near_plane", c_float), ("bg", c_float * 3)]


class Geom(ctypes.Structure):
    _fields_ = [("k", c_int32), ("pad", c_int32), ("rec", c_void_p), ("depth", c_void_p), ("rect", c_void_p),
                ("tiles", c_void_p), ("views", c_void_p)]


class SceneGrads(ctypes.Structure):
    _fields_ = [("accumulate", c_int32), ("flags", c_int32), ("means", c_void_p), ("scales", c_void_p), ("quats", c_void_p), ("opacities", c_void_p),
                ("sh", c_void_p), ("colors", c_void_p), ("freqs", c_void_p), ("weights", c_void_p),
                ("grad2d", c_void_p)]


class DensifyParams(ctypes.Structure):
    _fields_ = [("grad_threshold", c_float), ("percent_dense", c_float), ("scene_extent", c_float),
                ("min_opacity", c_float), ("max_world_frac", c_float), ("prune_big", c_int32),
                ("freq_reset", c_float), ("weight_reset", c_float), ("split_shrink", c_float),
                ("split_count", c_int32), ("abs_grad_threshold", c_float)]


class SceneOut(ctypes.Structure):
    _fields_ = [("n", c_int64), ("k", c_int32), ("sh_degree", c_int32), ("flags", c_int32), ("pad", c_int32),
                ("means", c_void_p), ("scales", c_void_p), ("quats", c_void_p), ("opacities", c_void_p),
                ("sh", c_void_p), ("colors", c_void_p), ("freqs", c_void_p), ("weights", c_void_p)]


_LIB: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise GabsplatError(HIP_ERROR, f"{LIB_PATH} not found: build it with `python -m paper_2508_05343_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.gabsplat_abi_version.restype = c_int32
    if L.gabsplat_abi_version() != ABI_VERSION:
        raise GabsplatError(INVALID_ARGUMENT, f"{LIB_PATH} has ABI version {L.gabsplat_abi_version()}, the binding "
                            f"expects {ABI_VERSION}: rebuild it with `python -m paper_2508_05343_amd.build`")
    L.gabsplat_status_string.restype = ctypes.c_char_p
    L.gabsplat_status_string.argtypes = [c_int32]
    L.gabsplat_record_floats.restype = c_int32
    L.gabsplat_record_floats.argtypes = [c_int32]
    L.gabsplat_row_floats.restype = c_int32
    L.gabsplat_row_floats.argtypes = [c_int32]
    L.gabsplat_pack_rows.restype = c_int32
    L.gabsplat_pack_rows.argtypes = [POINTER(Scene), c_void_p, c_void_p]
    L.gabsplat_grad2d_floats.restype = c_int32
    L.gabsplat_grad2d_floats.argtypes = [c_int32]
    L.gabsplat_grad2d_stride.restype = c_int32
    L.gabsplat_grad2d_stride.argtypes = [c_int32, c_int32]
    L.gabsplat_views_bytes.restype = c_size_t
    L.gabsplat_views_bytes.argtypes = [c_int32, c_int32]
    L.gabsplat_bin_sort_workspace_size.restype = c_size_t
    L.gabsplat_bin_sort_workspace_size.argtypes = [c_int64, c_int64, c_int64]
    L.gabsplat_check_device.restype = c_int32
    L.gabsplat_preprocess.restype = c_int32
    L.gabsplat_preprocess.argtypes = [POINTER(Scene), c_int32, POINTER(c_int32), POINTER(Camera), c_int32,
                                      POINTER(Geom), c_void_p]
    L.gabsplat_bin_sort.restype = c_int32
    L.gabsplat_bin_sort.argtypes = [POINTER(Geom), POINTER(Camera), c_int32, c_int64, c_void_p, c_size_t,
                                    c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
    L.gabsplat_render_fwd.restype = c_int32
    L.gabsplat_render_fwd.argtypes = [POINTER(Geom), c_void_p, c_void_p, POINTER(Camera), c_int32, c_void_p,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    L.gabsplat_render_bwd.restype = c_int32
    L.gabsplat_render_bwd.argtypes = [POINTER(Scene), c_int32, POINTER(c_int32), POINTER(Camera), c_int32,
                                      POINTER(Geom), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                      POINTER(SceneGrads), c_void_p, c_void_p]
    L.gabsplat_render_bwd_stages.restype = c_int32
    L.gabsplat_render_bwd_stages.argtypes = [POINTER(Scene), c_int32, POINTER(c_int32), POINTER(Camera), c_int32,
                                             POINTER(Geom), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                             POINTER(SceneGrads), c_void_p, c_int32, c_void_p]
    L.gabsplat_loss_workspace_size.restype = c_size_t
    L.gabsplat_loss_workspace_size.argtypes = [c_int32, c_int32, c_int32]
    L.gabsplat_loss_l1_dssim.restype = c_int32
    L.gabsplat_loss_l1_dssim.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_float, c_void_p,
                                         c_void_p, c_void_p, c_size_t, c_void_p]
    L.gabsplat_loss_l1_dssim_noalloc.restype = c_int32
    L.gabsplat_loss_l1_dssim_noalloc.argtypes = [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_float, c_void_p,
                                                 c_void_p, c_void_p]
    L.gabsplat_read_overflow.restype = c_int32
    L.gabsplat_read_overflow.argtypes = [c_void_p, c_void_p]
    L.gabsplat_densify_stats.restype = c_int32
    L.gabsplat_densify_stats.argtypes = [POINTER(Geom), POINTER(Camera), c_int32, c_int64, c_void_p, c_int32,
                                         c_void_p, c_void_p, c_void_p, c_void_p]
    L.gabsplat_densify_workspace_size.restype = c_size_t
    L.gabsplat_densify_workspace_size.argtypes = [c_int64]
    L.gabsplat_densify.restype = c_int32
    L.gabsplat_densify.argtypes = [POINTER(Scene), c_void_p, c_void_p, c_void_p, c_void_p, POINTER(DensifyParams),
                                   POINTER(SceneOut), c_int64, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   c_size_t, c_void_p]
    L.gabsplat_reset_frequency_weights.restype = c_int32
    L.gabsplat_reset_frequency_weights.argtypes = [POINTER(SceneOut), c_float, c_float, c_void_p]
    L.gabsplat_mip_filter3d_workspace_size.restype = c_size_t
    L.gabsplat_mip_filter3d_workspace_size.argtypes = [c_int64, c_int32]
    L.gabsplat_mip_filter3d.restype = c_int32
    L.gabsplat_mip_filter3d.argtypes = [c_void_p, c_int64, POINTER(Camera), c_int32, c_float, c_float, c_void_p,
                                        c_void_p, c_size_t, c_void_p]
    _LIB = L
    return L


def _check(status: int, what: str):
    if status != OK:
        msg = lib().gabsplat_status_string(status).decode()
        raise GabsplatError(status, f"{what}: {msg}")


def ptr(t) -> Optional[int]:
    """Raw device pointer of a tensor (None for None)."""
    if t is None:
        return None
    return int(t.data_ptr())


def stream_handle(stream=None) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream) or None


def _arr(ctype, items):
    items = list(items)
    return (ctype * max(1, len(items)))(*items)


# ------------------------------------------------------------------ helpers
def gabsplat_abi_version() -> int:
    return int(lib().gabsplat_abi_version())


def gabsplat_record_floats(k: int) -> int:
    return int(lib().gabsplat_record_floats(k))


def gabsplat_row_floats(k: int) -> int:
    return int(lib().gabsplat_row_floats(k))


def gabsplat_grad2d_floats(k: int) -> int:
    return int(lib().gabsplat_grad2d_floats(k))


def gabsplat_grad2d_stride(k: int, grad_flags: int) -> int:
    return int(lib().gabsplat_grad2d_stride(k, grad_flags))


def gabsplat_views_bytes(num_views: int, num_scenes: int) -> int:
    return int(lib().gabsplat_views_bytes(num_views, num_scenes))


def gabsplat_bin_sort_workspace_size(items: int, pair_capacity: int, total_tiles: int) -> int:
    return int(lib().gabsplat_bin_sort_workspace_size(items, pair_capacity, total_tiles))


def gabsplat_loss_workspace_size(c: int, h: int, w: int) -> int:
    return int(lib().gabsplat_loss_workspace_size(c, h, w))


def gabsplat_check_device():
    _check(lib().gabsplat_check_device(), "gabsplat_check_device")


# -------------------------------------------------------------- entry points
def gabsplat_preprocess(scenes: Sequence[Scene], scene_of_view: Optional[Sequence[int]], cams: Sequence[Camera],
                        geom: Geom, stream=None):
    sa = _arr(Scene, scenes)
    sv = None if scene_of_view is None else _arr(c_int32, scene_of_view)
    ca = _arr(Camera, cams)
    _check(lib().gabsplat_preprocess(sa, len(scenes), sv, ca, len(cams), ctypes.byref(geom),
                                     stream_handle(stream)), "gabsplat_preprocess")


def gabsplat_pack_rows(scene: Scene, rows, stream=None):
    _check(lib().gabsplat_pack_rows(ctypes.byref(scene), ptr(rows), stream_handle(stream)), "gabsplat_pack_rows")


def gabsplat_bin_sort(geom: Geom, cams: Sequence[Camera], items: int, ws, keys, vals, pair_capacity: int,
                      tile_ranges, d_num_pairs, d_overflow, stream=None):
    ca = _arr(Camera, cams)
    _check(lib().gabsplat_bin_sort(ctypes.byref(geom), ca, len(cams), items, ptr(ws), ws.numel() * ws.element_size(),
                                   ptr(keys), ptr(vals), pair_capacity, ptr(tile_ranges), ptr(d_num_pairs),
                                   ptr(d_overflow), stream_handle(stream)), "gabsplat_bin_sort")


def gabsplat_render_fwd(geom: Geom, vals, tile_ranges, cams: Sequence[Camera], image, final_T, n_contrib,
                        d_overflow, stream=None, eval_counts=None, freq_map=None):
    ca = _arr(Camera, cams)
    _check(lib().gabsplat_render_fwd(ctypes.byref(geom), ptr(vals), ptr(tile_ranges), ca, len(cams), ptr(image),
                                     ptr(final_T), ptr(n_contrib), ptr(eval_counts), ptr(freq_map),
                                     ptr(d_overflow), stream_handle(stream)), "gabsplat_render_fwd")


def gabsplat_render_bwd(scenes: Sequence[Scene], scene_of_view, cams: Sequence[Camera], geom: Geom, vals,
                        tile_ranges, final_T, n_contrib, dl_dimage, grads: Sequence[SceneGrads], d_overflow,
                        stream=None):
    sa = _arr(Scene, scenes)
    sv = None if scene_of_view is None else _arr(c_int32, scene_of_view)
    ca = _arr(Camera, cams)
    ga = _arr(SceneGrads, grads)
    _check(lib().gabsplat_render_bwd(sa, len(scenes), sv, ca, len(cams), ctypes.byref(geom), ptr(vals),
                                     ptr(tile_ranges), ptr(final_T), ptr(n_contrib), ptr(dl_dimage), ga,
                                     ptr(d_overflow), stream_handle(stream)), "gabsplat_render_bwd")


def gabsplat_render_bwd_stages(scenes: Sequence[Scene], scene_of_view, cams: Sequence[Camera], geom: Geom, vals,
                               tile_ranges, final_T, n_contrib, dl_dimage, grads: Sequence[SceneGrads], d_overflow,
                               stages: int, stream=None):
    sa = _arr(Scene, scenes)
    sv = None if scene_of_view is None else _arr(c_int32, scene_of_view)
    ca = _arr(Camera, cams)
    ga = _arr(SceneGrads, grads)
    _check(lib().gabsplat_render_bwd_stages(sa, len(scenes), sv, ca, len(cams), ctypes.byref(geom), ptr(vals),
                                            ptr(tile_ranges), ptr(final_T), ptr(n_contrib), ptr(dl_dimage), ga,
                                            ptr(d_overflow), int(stages), stream_handle(stream)),
           "gabsplat_render_bwd_stages")


def _loss_args(x, y, d_loss, dl_dx):
    """Layout checks of the loss bindings: x, y and dl_dx contiguous float32
    [channels][H][W] device tensors of one shape on one device, d_loss at least
    one float32 there."""
    import torch
    for name, t in (("x", x), ("y", y), ("dl_dx", dl_dx), ("d_loss", d_loss)):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 device tensor")
        if t.device != x.device:
            raise ValueError(f"{name} is on {t.device}, x on {x.device}")
    if x.dim() != 3 or y.shape != x.shape or dl_dx.shape != x.shape:
        raise ValueError(f"x, y and dl_dx must share one [channels, H, W] shape, got {tuple(x.shape)}, "
                         f"{tuple(y.shape)}, {tuple(dl_dx.shape)}")
    if d_loss.numel() < 1:
        raise ValueError("d_loss must hold one float")
    return x.shape


def gabsplat_loss_l1_dssim(x, y, lam: float, d_loss, dl_dx, ws, stream=None):
    c, h, w = _loss_args(x, y, d_loss, dl_dx)
    _check(lib().gabsplat_loss_l1_dssim(ptr(x), ptr(y), c, h, w, float(lam), ptr(d_loss), ptr(dl_dx), ptr(ws),
                                        ws.numel() * ws.element_size(), stream_handle(stream)),
           "gabsplat_loss_l1_dssim")


def gabsplat_loss_l1_dssim_noalloc(x, y, lam: float, d_loss, dl_dx, stream=None):
    c, h, w = _loss_args(x, y, d_loss, dl_dx)
    _check(lib().gabsplat_loss_l1_dssim_noalloc(ptr(x), ptr(y), c, h, w, float(lam), ptr(d_loss), ptr(dl_dx),
                                                stream_handle(stream)),
           "gabsplat_loss_l1_dssim_noalloc")


def gabsplat_densify_stats(geom: Geom, cams: Sequence[Camera], n: int, grad2d, grad_flags: int, accum, accum_abs,
                           denom, stream=None):
    ca = _arr(Camera, cams)
    _check(lib().gabsplat_densify_stats(ctypes.byref(geom), ca, len(cams), n, ptr(grad2d), grad_flags, ptr(accum),
                                        ptr(accum_abs), ptr(denom), stream_handle(stream)), "gabsplat_densify_stats")


def gabsplat_densify_workspace_size(n: int) -> int:
    return int(lib().gabsplat_densify_workspace_size(n))


def gabsplat_densify(scene_in: Scene, accum, denom, accum_abs, normals, params: DensifyParams, out: SceneOut,
                     out_capacity: int, src_index, tag, d_n_out, d_overflow, ws, stream=None):
    _check(lib().gabsplat_densify(ctypes.byref(scene_in), ptr(accum), ptr(denom), ptr(accum_abs), ptr(normals),
                                  ctypes.byref(params), ctypes.byref(out), out_capacity, ptr(src_index), ptr(tag),
                                  ptr(d_n_out), ptr(d_overflow), ptr(ws), ws.numel() * ws.element_size(),
                                  stream_handle(stream)), "gabsplat_densify")


def gabsplat_reset_frequency_weights(scene: SceneOut, weight_value: float, opacity_cap: float, stream=None):
    _check(lib().gabsplat_reset_frequency_weights(ctypes.byref(scene), float(weight_value), float(opacity_cap),
                                                  stream_handle(stream)), "gabsplat_reset_frequency_weights")


def gabsplat_mip_filter3d_workspace_size(n: int, num_cams: int) -> int:
    return int(lib().gabsplat_mip_filter3d_workspace_size(n, num_cams))


def gabsplat_mip_filter3d(means, n: int, cams: Sequence[Camera], s: float, margin: float, filter3d, ws,
                          stream=None):
    ca = _arr(Camera, cams)
    _check(lib().gabsplat_mip_filter3d(ptr(means), n, ca, len(cams), float(s), float(margin), ptr(filter3d), ptr(ws),
                                       ws.numel() * ws.element_size(), stream_handle(stream)), "gabsplat_mip_filter3d")


def gabsplat_read_overflow(d_overflow, stream=None) -> bool:
    """True if the last bin sort overflowed its pair capacity (synchronises)."""
    st = lib().gabsplat_read_overflow(ptr(d_overflow), stream_handle(stream))
    if st == CAPACITY_EXCEEDED:
        return True
    _check(st, "gabsplat_read_overflow")
    return False
