"""CPU reference ("oracle") for the 3D Gabor splatting rasterizer.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import or call
this module; it exists so that tests, the smoke check and the CPU-baseline leg
of the benchmark can check the GPU path against a plain, slow, obviously
correct definition.  It shares no code with the GPU path.

Everything is computed in float64 with plain PyTorch CPU ops, except the
three decisions the method takes on float32 data (the depth key, the near-plane
cull and the opacity cull), which are taken on float32 values here as well.
The exact derivative of the whole forward is obtained with torch.autograd on
this float64 definition (the backward is therefore not a second hand-written
formula that could share a mistake with the forward).

Per-primitive steps follow the paper:
  * 3D envelope and covariance Sigma = R S S^T R^T (Sec. 3.1, Eq. 3d_gaussian).
  * Gabor filter bank G(x) [(1 - sum w) + sum w cos(2 pi f^T (x - mu))]
    (Sec. 3.2, the 3D Gabor-based primitive).
  * EWA projection Sigma' = J W Sigma W^T J^T with the 2x2 block as the 2D
    covariance (Sec. 3.1).
  * Frequency projection f_proj = (JW)^{-T} f (Sec. 3.3.1; supplementary A.1)
    followed by the z-integration f2d = f_proj,xy - (S_xy,z / S_zz) f_proj,z
    with S the inverse ray-space covariance (Sec. 3.3.2; supplementary A.2).
    Written out, this equals (T Sigma T^T)^{-1} T Sigma f where T is the first
    two rows of JW, for any full-rank completion of J; that closed form is
    what is evaluated here (tests check it against the paper's two-step form).
  * 2D Gabor primitive and front-to-back alpha blending (Sec. 3.3.2 and 3.3.3).
The per-pixel blend takes every visible primitive sorted by (fp32 depth,
index): alpha = min(0.99, o G B); skip if alpha < 1/255; stop without blending
when T (1 - alpha) < 1e-4; background added with the final transmittance.

Readings where the paper is silent (tile rasterizer conventions adopted from
3DGS, which the paper says it adapts in Sec. 3.3.3): 0.3 px^2 dilation of the
2D covariance, 1.3x guard band on the Jacobian's evaluation point, near plane
0.2 on camera z, opacity-aware support radius sqrt(2 ln(255 o)), pixel centres
at (px + 0.5, py + 0.5), real spherical harmonics of degree <= 3 with +0.5 and
a clamp at 0, 16x16 tiles, ties in depth broken by primitive index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

DT = torch.float64
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
DILATION = 0.3
TILE = 16
# Plug-in anti-aliasing (Mip-Splatting, combined with 3DGabSplat in Sec. 4.1
# and Table 1): the 2D filter replaces the dilation by a Gaussian of variance
# 0.1 px^2 (a one-pixel box) and rescales the opacity so that the envelope's
# integral is kept; the ratio det(S) / det(S + 0.1 I) is floored (a reading).
MIP2D_VARIANCE = 0.1
MIP2D_MIN_RATIO = 1e-6


# --------------------------------------------------------------------------
# input marshalling (scene / camera objects -> fp64 tensors)
# --------------------------------------------------------------------------
def scene_tensors(scene, requires_grad: bool = False) -> Dict[str, torch.Tensor]:
    """fp64 leaf tensors for the activated primitive attributes."""
    out = {}
    for name in ("means", "scales", "quats", "opacities", "freqs", "weights", "colors", "sh"):
        a = getattr(scene, name)
        if a is None:
            continue
        t = torch.tensor(np.asarray(a, np.float64), dtype=DT)
        if requires_grad:
            t.requires_grad_(True)
        out[name] = t
    return out


def camera_tensors(cam) -> Dict[str, object]:
    return dict(
        R=torch.tensor(np.asarray(cam.R, np.float64), dtype=DT),
        t=torch.tensor(np.asarray(cam.t, np.float64), dtype=DT),
        eye=torch.tensor(np.asarray(cam.eye, np.float64), dtype=DT),
        fx=float(cam.fx), fy=float(cam.fy), cx=float(cam.cx), cy=float(cam.cy),
        W=int(cam.width), H=int(cam.height), near=float(cam.near),
        bg=torch.tensor(cam.bg, dtype=DT),
    )


# --------------------------------------------------------------------------
# 3D primitive (Sec. 3.1 / 3.2)
# --------------------------------------------------------------------------
def quat_to_rotmat(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrix of the (normalised) quaternion (w, x, y, z)."""
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    r0 = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1)
    r1 = torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1)
    r2 = torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)
    return torch.stack([r0, r1, r2], -2)


def covariance_3d(scales: torch.Tensor, quats: torch.Tensor) -> torch.Tensor:
    """Sigma = R S S^T R^T with S = diag(scales) (Sec. 3.1)."""
    M = quat_to_rotmat(quats) * scales[..., None, :]
    return M @ M.transpose(-1, -2)


# --------------------------------------------------------------------------
# real spherical harmonics (colour), written from the closed form
# Y_l^m ~ K_l^m * {Re, Im}((x + i y)^|m|) * d^|m| P_l / dz^|m|  (no Condon-Shortley phase)
# --------------------------------------------------------------------------
def _sh_norm(l: int, m: int) -> float:
    return math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - abs(m)) / math.factorial(l + abs(m)))


def _legendre_derivative_coeffs(l: int, m: int) -> np.ndarray:
    """Power-series coefficients (ascending) of d^m/dz^m P_l(z)."""
    c = np.polynomial.legendre.leg2poly(np.eye(l + 1)[l])
    for _ in range(m):
        c = np.polynomial.polynomial.polyder(c)
    return c


def sh_basis(dirs: torch.Tensor, degree: int) -> torch.Tensor:
    """[..., (degree+1)^2] real SH basis at unit directions dirs [..., 3];
    order l = 0..degree, m = -l..l."""
    x, y, z = dirs.unbind(-1)
    A = [torch.ones_like(x)]
    B = [torch.zeros_like(x)]
    for m in range(1, degree + 1):  # Re / Im of (x + i y)^m = (x + i y)(A + i B)
        a_prev, b_prev = A[-1], B[-1]
        A.append(x * a_prev - y * b_prev)
        B.append(x * b_prev + y * a_prev)
    out = []
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            coeffs = _legendre_derivative_coeffs(l, abs(m))
            q = torch.zeros_like(z)
            for c in coeffs[::-1]:  # Horner
                q = q * z + float(c)
            k = _sh_norm(l, m)
            if m > 0:
                out.append(math.sqrt(2.0) * k * A[m] * q)
            elif m < 0:
                out.append(math.sqrt(2.0) * k * B[-m] * q)
            else:
                out.append(k * q)
    return torch.stack(out, -1)


def sh_to_rgb(sh: torch.Tensor, means: torch.Tensor, eye: torch.Tensor) -> torch.Tensor:
    """Colour = max(0, sum_d sh[d] Y_d(dir) + 0.5), dir = (mu - eye)/|mu - eye|."""
    d = means - eye
    d = d / torch.linalg.norm(d, dim=-1, keepdim=True)
    deg = int(round(math.sqrt(sh.shape[-2]))) - 1
    Y = sh_basis(d, deg)  # [n, D]
    rgb = torch.einsum("nd,ndc->nc", Y, sh) + 0.5
    return torch.clamp(rgb, min=0.0)


# --------------------------------------------------------------------------
# projection (Sec. 3.1 EWA, Sec. 3.3 frequency projection + z-integration)
# --------------------------------------------------------------------------
def depth_fp32(means_f32: np.ndarray, R_f32: np.ndarray, t_f32: np.ndarray) -> np.ndarray:
    """Camera-space z as a float32 key, fixed evaluation order, one IEEE
    rounding per operation: ((r20 x + r21 y) + r22 z) + t2."""
    m = np.asarray(means_f32, np.float32)
    r = np.asarray(R_f32, np.float32)
    t2 = np.float32(np.asarray(t_f32, np.float32)[2])
    a = r[2, 0] * m[:, 0]
    b = r[2, 1] * m[:, 1]
    c = r[2, 2] * m[:, 2]
    return ((a + b) + c) + t2


def filtered_envelope(scales: torch.Tensor, opacities: torch.Tensor, variances):
    """Mip-Splatting's 3D smoothing filter applied to the Gaussian envelope:
    the envelope o exp(-x^T Sigma^-1 x / 2) convolved with the normalised
    isotropic Gaussian of variance v is o' exp(-x^T Sigma'^-1 x / 2) with
    Sigma' = Sigma + v I -- for Sigma = R diag(s^2) R^T, the scales
    sqrt(s^2 + v) -- and o' = o sqrt(det Sigma / det Sigma') = o prod_j s_j /
    sqrt(s_j^2 + v).  Returns (filtered scales, filtered opacities)."""
    fv = torch.as_tensor(np.asarray(variances, np.float64), dtype=DT)
    s_f = torch.sqrt(scales * scales + fv[:, None])
    return s_f, opacities * torch.prod(scales / s_f, -1)


@dataclass
class Projected:
    visible: torch.Tensor       # [n] bool
    depth32: np.ndarray         # [n] float32
    mu2d: torch.Tensor          # [n,2]
    cov2d_raw: torch.Tensor     # [n,2,2]
    conic: torch.Tensor         # [n,3] (xx, xy, yy) of (cov2d_raw + 0.3 I)^-1
    opac: torch.Tensor          # [n]
    rgb: torch.Tensor           # [n,3]
    f2d: torch.Tensor           # [n,K,2] cycles per pixel
    w: torch.Tensor             # [n,K] weights of the cosine terms (attenuated if requested)
    rect: np.ndarray            # [n,4] int64 tile rect x0,y0,x1,y1 (exclusive)
    tiles: np.ndarray           # [n] tiles touched (0 if invisible)
    fragile_rect: np.ndarray    # [n] bool: rect boundary within 2e-3 px of a pixel centre
    fragile_prim: np.ndarray    # [n] bool: ill-conditioned 2D frequency solve


def project(p: Dict[str, torch.Tensor], cam: Dict[str, object], scene_f32=None,
            attenuation: bool = False, mip2d: bool = False, filter3d=None) -> Projected:
    """Per-primitive projection.  ``p`` holds fp64 tensors (possibly requiring
    grad); ``scene_f32`` supplies the float32 means/opacities for the fp32
    decisions (defaults to rounding p's values, which are exact copies).

    attenuation=True keeps the factor the z-integration of supplementary A.2
    produces for every cosine term and the paper's final 2D primitive drops:
    w_k -> w_k exp(-2 pi^2 v_k), v_k = f_k^T Sigma f_k - (T Sigma f_k)^T
    (T Sigma T^T)^-1 (T Sigma f_k), the variance of f_k . x along the ray
    given the image-plane point (the DC weight 1 - sum w is unchanged).

    filter3d (per-primitive variances, see mip_filter3d) convolves the Gaussian
    envelope with an isotropic 3D Gaussian of that variance: Sigma -> Sigma +
    v I, i.e. every scale s -> sqrt(s^2 + v), and the opacity is multiplied by
    sqrt(det Sigma / det(Sigma + v I)) = prod_j s_j / sqrt(s_j^2 + v), which
    keeps the envelope's integral.  mip2d replaces the 0.3 px^2 dilation by the
    2D filter (variance 0.1 px^2, opacity times sqrt(det S / det(S + 0.1 I)),
    S the undilated 2D covariance).  Both act on the envelope only: the 3D
    frequencies and weights are left as they are (the plug-in reading: the
    Gaussian of the other method is replaced by the Gabor primitive and nothing
    else changes), and the frequency projection, like every other use of
    Sigma, sees the filtered covariance.  The near and opacity culls stay on
    the input values; a primitive whose filtered opacity is at most 1/255 is
    invisible."""
    R, t = cam["R"], cam["t"]
    fx, fy, cx, cy = cam["fx"], cam["fy"], cam["cx"], cam["cy"]
    W, H = cam["W"], cam["H"]
    means = p["means"]
    n = means.shape[0]
    if scene_f32 is None:
        m32 = means.detach().numpy().astype(np.float32)
        o32 = p["opacities"].detach().numpy().astype(np.float32)
    else:
        m32, o32 = np.asarray(scene_f32.means, np.float32), np.asarray(scene_f32.opacities, np.float32)
    R32 = R.numpy().astype(np.float32)
    t32 = t.numpy().astype(np.float32)

    # camera space (W of the paper is [R | t])
    tc = means @ R.T + t
    tx, ty, tz = tc.unbind(-1)
    depth32 = depth_fp32(m32, R32, t32)
    scales, opac = p["scales"], p["opacities"]
    if filter3d is not None:
        scales, opac = filtered_envelope(scales, opac, filter3d)
    in_front = torch.from_numpy(depth32 > np.float32(cam["near"]))
    opac_ok = torch.from_numpy(o32 * np.float32(255.0) > np.float32(1.0))

    # keep culled entries finite: evaluate them at a harmless depth
    tz_safe = torch.where(in_front, tz, torch.ones_like(tz))
    mu2d = torch.stack([fx * tx / tz_safe + cx, fy * ty / tz_safe + cy], -1)

    # Jacobian of the perspective map at the guard-band-clamped point
    lo_x, hi_x = (-0.15 * W - cx) / fx, (1.15 * W - cx) / fx
    lo_y, hi_y = (-0.15 * H - cy) / fy, (1.15 * H - cy) / fy
    txc = torch.clamp(tx / tz_safe, lo_x, hi_x) * tz_safe
    tyc = torch.clamp(ty / tz_safe, lo_y, hi_y) * tz_safe
    zero = torch.zeros_like(tz_safe)
    J2 = torch.stack([
        torch.stack([fx / tz_safe, zero, -fx * txc / (tz_safe * tz_safe)], -1),
        torch.stack([zero, fy / tz_safe, -fy * tyc / (tz_safe * tz_safe)], -1),
    ], -2)                                   # [n,2,3]
    T = J2 @ R                               # first two rows of J W
    Sig = covariance_3d(scales, p["quats"])
    cov_raw = T @ Sig @ T.transpose(-1, -2)  # [n,2,2]
    dil = MIP2D_VARIANCE if mip2d else DILATION
    a = cov_raw[:, 0, 0] + dil
    b = cov_raw[:, 0, 1]
    c = cov_raw[:, 1, 1] + dil
    det = a * c - b * b
    det_ok = det > 0
    det_safe = torch.where(det_ok, det, torch.ones_like(det))
    conic = torch.stack([c / det_safe, -b / det_safe, a / det_safe], -1)

    # 2D frequencies: f2d_k = (T Sigma T^T)^-1 (T Sigma f_k)
    K = p["weights"].shape[1]
    ra, rb, rc = cov_raw[:, 0, 0], cov_raw[:, 0, 1], cov_raw[:, 1, 1]
    det_raw = ra * rc - rb * rb
    scale_raw = ra * rc
    cond_bad = (det_raw.detach() <= 1e-6 * scale_raw.detach()) | (det_raw.detach() <= 0)
    det_raw_safe = torch.where(det_raw > 0, det_raw, torch.ones_like(det_raw))
    if K > 0:
        g = torch.einsum("nij,njk,nck->nci", T, Sig, p["freqs"])   # [n,K,2] = T Sigma f_k
        fxp = (rc[:, None] * g[..., 0] - rb[:, None] * g[..., 1]) / det_raw_safe[:, None]
        fyp = (-rb[:, None] * g[..., 0] + ra[:, None] * g[..., 1]) / det_raw_safe[:, None]
        f2d = torch.stack([fxp, fyp], -1)
        f2d = torch.where((det_raw > 0)[:, None, None], f2d, torch.zeros_like(f2d))
        w_cos = p["weights"]
        if attenuation:
            fSf = torch.einsum("nck,nkl,ncl->nc", p["freqs"], Sig, p["freqs"])
            v = fSf - (g[..., 0] * fxp + g[..., 1] * fyp)  # g^T (T Sigma T^T)^-1 g = g . f2d
            v = torch.where((det_raw > 0)[:, None], v, fSf)
            w_cos = p["weights"] * torch.exp(-2.0 * math.pi ** 2 * v)
    else:
        f2d = torch.zeros((n, 0, 2), dtype=DT)
        w_cos = p["weights"]

    if mip2d:
        det_r = cov_raw[:, 0, 0] * cov_raw[:, 1, 1] - cov_raw[:, 0, 1] ** 2
        ratio = torch.clamp(det_r / det_safe, min=MIP2D_MIN_RATIO)
        opac = opac * torch.sqrt(ratio)

    # colour
    if "sh" in p:
        rgb = sh_to_rgb(p["sh"], means, cam["eye"])
    else:
        rgb = p["colors"]

    # support: o * G >= 1/255 inside the ellipse d^T conic d <= 2 ln(255 o)
    with torch.no_grad():
        o64 = opac.detach()
        kk = torch.sqrt(torch.clamp(2.0 * torch.log(255.0 * o64), min=0.0))
        rx = kk * torch.sqrt(torch.clamp(a.detach(), min=0.0))
        ry = kk * torch.sqrt(torch.clamp(c.detach(), min=0.0))
        mx, my = mu2d[:, 0].detach(), mu2d[:, 1].detach()
        bx0, bx1 = (mx - rx - 0.5).numpy(), (mx + rx - 0.5).numpy()
        by0, by1 = (my - ry - 0.5).numpy(), (my + ry - 0.5).numpy()
        with np.errstate(invalid="ignore", over="ignore"):
            px0 = np.maximum(np.ceil(bx0), 0)
            px1 = np.minimum(np.floor(bx1), W - 1)
            py0 = np.maximum(np.ceil(by0), 0)
            py1 = np.minimum(np.floor(by1), H - 1)
        ok = (px0 <= px1) & (py0 <= py1) & np.isfinite(bx0) & np.isfinite(by0)
        vis = in_front.numpy() & opac_ok.numpy() & det_ok.numpy() & ok
        filtered = filter3d is not None or mip2d
        if filtered:
            vis &= (255.0 * o64).numpy() > 1.0
        rect = np.zeros((n, 4), np.int64)
        rect[vis, 0] = (px0[vis] // TILE).astype(np.int64)
        rect[vis, 1] = (py0[vis] // TILE).astype(np.int64)
        rect[vis, 2] = (px1[vis] // TILE).astype(np.int64) + 1
        rect[vis, 3] = (py1[vis] // TILE).astype(np.int64) + 1
        tiles = np.where(vis, (rect[:, 2] - rect[:, 0]) * (rect[:, 3] - rect[:, 1]), 0)

        def near_int(v):
            with np.errstate(invalid="ignore"):
                return np.abs(v - np.round(v)) < 2e-3
        fr = vis & (near_int(bx0) | near_int(bx1) | near_int(by0) | near_int(by1))
        if filtered:  # the filtered-opacity test taken in fp32 may differ near 1/255
            fr |= in_front.numpy() & opac_ok.numpy() & (np.abs(255.0 * o64.numpy() - 1.0) < 1e-4)
        fp = vis & cond_bad.numpy()
    pr = Projected(visible=torch.from_numpy(vis), depth32=depth32, mu2d=mu2d, cov2d_raw=cov_raw,
                   conic=conic, opac=opac, rgb=rgb, f2d=f2d, w=w_cos,
                   rect=rect, tiles=tiles.astype(np.int64), fragile_rect=fr, fragile_prim=fp)
    pr.w_dc = 1.0 - p["weights"].sum(-1)  # DC weight, never attenuated
    return pr


# --------------------------------------------------------------------------
# depth order, tile binning and the (tile, depth) key sort
# --------------------------------------------------------------------------
def depth_order(depth32: np.ndarray, visible: np.ndarray) -> np.ndarray:
    """Indices of visible primitives sorted by (fp32 depth bit pattern, index)."""
    idx = np.nonzero(np.asarray(visible))[0]
    bits = np.asarray(depth32, np.float32).view(np.uint32)[idx]
    return idx[np.lexsort((idx, bits))]


def bin_sort(rect: np.ndarray, depth32: np.ndarray, visible: np.ndarray, tiles_x: int,
             num_tiles: int, tile_offset: int = 0, index_offset: int = 0):
    """Emit one (key, value) per (primitive, overlapped tile) in primitive
    order and, within a primitive, row-major tile order; key = tile << 32 |
    depth bits, value = primitive index.  Sort stably by key (library stable
    sort) and derive the [start, end) range of every tile; empty tiles get
    (0, 0).  Returns keys uint64, vals uint32, ranges [num_tiles, 2] uint32."""
    keys, vals = [], []
    bits = np.asarray(depth32, np.float32).view(np.uint32).astype(np.uint64)
    for i in np.nonzero(np.asarray(visible))[0]:
        x0, y0, x1, y1 = (int(v) for v in rect[i])
        for ty in range(y0, y1):
            for tx in range(x0, x1):
                tile = tile_offset + ty * tiles_x + tx
                keys.append((np.uint64(tile) << np.uint64(32)) | bits[i])
                vals.append(index_offset + i)
    keys = np.asarray(keys, np.uint64)
    vals = np.asarray(vals, np.uint32)
    order = np.argsort(keys, kind="stable")
    keys, vals = keys[order], vals[order]
    ranges = np.zeros((num_tiles, 2), np.uint32)
    tl = (keys >> np.uint64(32)).astype(np.int64) - tile_offset
    for pos in range(len(tl)):
        t_ = tl[pos]
        if pos == 0 or tl[pos - 1] != t_:
            ranges[t_, 0] = pos
        if pos == len(tl) - 1 or tl[pos + 1] != t_:
            ranges[t_, 1] = pos + 1
    return keys, vals, ranges


# --------------------------------------------------------------------------
# per-pixel blending (Sec. 3.3.2 2D Gabor primitive, Sec. 3.3.3 blend)
# --------------------------------------------------------------------------
@dataclass
class PixelResult:
    color: torch.Tensor      # [P,3]
    final_T: torch.Tensor    # [P]
    last_id: np.ndarray      # [P] primitive index of the last blended primitive, -1 if none
    n_blended: np.ndarray    # [P] number of blended primitives
    fragile: np.ndarray      # [P] bool
    freq_map: Optional[torch.Tensor] = None  # [P] blended sum_k w_k |f2d_k| (cycles/px)
    n_fragile: Optional[np.ndarray] = None   # [P] number of fragile decisions up to the stop
    fragile_bound: Optional[np.ndarray] = None  # [P] their largest effect, in units of the colour span
    # [P, m] the fragile skip decisions (alpha within tolerance of 1/255) and
    # stop decisions (T (1 - alpha) within tolerance of 1e-4) up to the stop
    frag_alpha: Optional[np.ndarray] = None
    frag_stop: Optional[np.ndarray] = None


# the per-primitive 2D record the blend reads (Projected attributes)
RECORD_FIELDS = ("mu2d", "conic", "opac", "rgb", "f2d", "w", "w_dc")

def blend_pixels(pr: Projected, cand: np.ndarray, px: torch.Tensor, py: torch.Tensor,
                 bg: torch.Tensor, tau_alpha=1e-4, tau_T=1e-3, mu: Optional[torch.Tensor] = None,
                 rec: Optional[Dict[str, torch.Tensor]] = None, flip_alpha: Optional[np.ndarray] = None,
                 flip_stop: Optional[np.ndarray] = None) -> PixelResult:
    """Blend the candidates ``cand`` (already sorted front to back) at the
    sample points (px, py), vectorised over pixels and candidates.

    ``rec`` (optional) gives every pixel its own copy of some of the
    candidates' 2D record fields (RECORD_FIELDS; each [P, m, ...], same
    values), so that a backward pass returns each pixel's share of their
    gradient separately; ``mu`` ([P, m, 2]) is the same for the means alone.
    ``flip_alpha`` / ``flip_stop`` ([P, m] bool, optional) take the marked
    decisions the other way: a marked candidate is skipped where the rule
    blends it and blended where the rule skips it (flip_alpha), or the walk
    stops at a marked candidate where the rule walks on, and walks on (blending
    it) where the rule stops (flip_stop).  They describe the other outcome of a
    decision taken within rounding of its threshold."""
    P = px.shape[0]
    m = len(cand)
    if m == 0:
        col = bg[None, :].expand(P, 3).clone()
        return PixelResult(col, torch.ones(P, dtype=DT), -np.ones(P, np.int64),
                           np.zeros(P, np.int64), np.zeros(P, bool), torch.zeros(P, dtype=DT), np.zeros(P, np.int64),
                           np.zeros(P), np.zeros((P, 0), bool), np.zeros((P, 0), bool))
    ci = torch.from_numpy(np.asarray(cand, np.int64))
    rec = dict(rec or {})
    if mu is not None:
        rec["mu2d"] = mu

    def field(name):
        # [P or 1, m, ...]
        return rec[name] if name in rec else getattr(pr, name)[ci][None]
    mu_ = field("mu2d")
    con = field("conic")
    dx = px[:, None] - mu_[..., 0]
    dy = py[:, None] - mu_[..., 1]
    G = torch.exp(-0.5 * (con[..., 0] * dx * dx + 2.0 * con[..., 1] * dx * dy
                          + con[..., 2] * dy * dy))
    w = field("w")
    if w.shape[-1] > 0:
        f = field("f2d")
        phase = f[..., 0] * dx[..., None] + f[..., 1] * dy[..., None]
        Bk = field("w_dc") + (w * torch.cos(2.0 * math.pi * phase)).sum(-1)
    else:
        Bk = torch.ones_like(G)
    a_raw = field("opac") * G * Bk
    alpha = torch.clamp(a_raw, max=ALPHA_MAX)
    with torch.no_grad():
        valid = alpha >= ALPHA_MIN
        if flip_alpha is not None:
            valid = valid ^ torch.from_numpy(np.asarray(flip_alpha, bool))
        one_m = torch.where(valid, 1.0 - alpha, torch.ones_like(alpha))
        T_after = torch.cumprod(one_m, dim=1)
        if flip_stop is None:
            keep = valid & (T_after >= T_MIN)
        else:
            # a stop event ends the walk; no record at or after it is blended
            stop_ev = valid & ((T_after < T_MIN) ^ torch.from_numpy(np.asarray(flip_stop, bool)))
            before = (torch.cumsum(stop_ev.to(torch.int64), 1) - stop_ev.to(torch.int64)) == 0
            keep = valid & ~stop_ev & before
    factor = torch.where(keep, 1.0 - alpha, torch.ones_like(alpha))
    T_incl = torch.cumprod(factor, dim=1)
    T_before = torch.cat([torch.ones((P, 1), dtype=DT), T_incl[:, :-1]], 1)
    wgt = torch.where(keep, alpha * T_before, torch.zeros_like(alpha))
    rgb = field("rgb")
    if rgb.shape[0] == 1:
        blended = wgt @ rgb[0]
    else:
        blended = (wgt[..., None] * rgb).sum(1)
    color = blended + T_incl[:, -1:] * bg[None, :]
    # frequency map (supplementary C): per primitive sum_k w_k |f2d_k|, blended like a colour
    phi = (pr.w[ci] * torch.linalg.norm(pr.f2d[ci], dim=-1)).sum(-1) if pr.w.shape[1] else torch.zeros(m, dtype=DT)
    fmap = wgt @ phi
    with torch.no_grad():
        kn = keep.numpy()
        n_bl = kn.sum(1)
        has = kn.any(1)
        last_pos = np.where(has, m - 1 - np.argmax(kn[:, ::-1], axis=1), -1)
        last_id = np.where(has, np.asarray(cand)[np.maximum(last_pos, 0)], -1)
        # fragility: decisions within tolerance of their thresholds, up to the stop point
        vn, Ta = valid.numpy(), T_after.numpy()
        stopped = vn & (Ta < T_MIN)
        stop_pos = np.where(stopped.any(1), np.argmax(stopped, axis=1), m - 1)
        upto = np.arange(m)[None, :] <= stop_pos[:, None]
        ar = a_raw.detach().numpy()
        fa = np.abs(ar - ALPHA_MIN) <= tau_alpha * ALPHA_MIN
        ft = vn & (np.abs(Ta - T_MIN) <= tau_T * T_MIN)
        fprim = (pr.fragile_prim[np.asarray(cand)][None, :]) & (ar >= ALPHA_MIN * (1 - tau_alpha))
        n_frag = ((fa | ft | fprim) & upto).sum(1)
        fragile = n_frag > 0
        # how far each fragile decision can move the pixel, in units of the
        # colour span max|c - bg|: with T_j the transmittance before record j
        # on the walk, blending or skipping j changes the colour by
        # alpha_j T_j (c_j - C_behind) (at most 2 alpha_j T_j span), and
        # stopping at j instead of walking on by T_j (bg - C_behind) (at most
        # T_j span); an ill-conditioned frequency solve can move alpha_j
        # anywhere in [0, 0.99] (at most 2 T_j span)
        Tb = np.concatenate([np.ones((P, 1)), Ta[:, :-1]], 1)
        al = alpha.detach().numpy()
        fb = (fa * 2.0 * np.clip(al, 0.0, None) * Tb + ft * Tb + fprim * 2.0 * Tb) * upto
        frag_bound = fb.sum(1)
    return PixelResult(color, T_incl[:, -1], last_id.astype(np.int64), n_bl.astype(np.int64), fragile, fmap,
                       n_frag.astype(np.int64), frag_bound, fa & upto, ft & upto)


def blend_pixel_loop(pr: Projected, cand: Sequence[int], x: float, y: float, bg) -> tuple:
    """The same blend for ONE pixel as a literal sequential loop (small cases
    only).  Returns (rgb list, final T, last primitive id, count)."""
    T = 1.0
    C = [0.0, 0.0, 0.0]
    last, cnt = -1, 0
    for i in cand:
        mx, my = float(pr.mu2d[i, 0]), float(pr.mu2d[i, 1])
        a, b, c = (float(v) for v in pr.conic[i])
        dx, dy = x - mx, y - my
        G = math.exp(-0.5 * (a * dx * dx + 2 * b * dx * dy + c * dy * dy))
        Bv = float(pr.w_dc[i])
        for k in range(pr.w.shape[1]):
            wk = float(pr.w[i, k])
            ph = float(pr.f2d[i, k, 0]) * dx + float(pr.f2d[i, k, 1]) * dy
            Bv += wk * math.cos(2 * math.pi * ph)
        alpha = min(ALPHA_MAX, float(pr.opac[i]) * G * Bv)
        if alpha < ALPHA_MIN:
            continue
        if T * (1.0 - alpha) < T_MIN:
            break
        for ch in range(3):
            C[ch] += float(pr.rgb[i, ch]) * alpha * T
        T *= 1.0 - alpha
        last, cnt = i, cnt + 1
    return [C[ch] + T * float(bg[ch]) for ch in range(3)], T, last, cnt


# --------------------------------------------------------------------------
# whole-image drivers
# --------------------------------------------------------------------------
@dataclass
class Image:
    color: torch.Tensor    # [3,H,W]
    final_T: torch.Tensor  # [H,W]
    last_id: np.ndarray    # [H,W]
    n_blended: np.ndarray  # [H,W]
    fragile: np.ndarray    # [H,W]
    freq_map: Optional[torch.Tensor] = None  # [H,W]
    n_fragile: Optional[np.ndarray] = None   # [H,W] fragile decisions per pixel
    # max over visible primitives and channels of |colour - background|
    colour_span: float = 0.0
    # [H,W] largest change of the pixel that its fragile decisions can cause,
    # in units of colour_span (PixelResult.fragile_bound)
    fragile_bound: Optional[np.ndarray] = None


def _tile_pixels(tx, ty, W, H):
    xs = np.arange(tx * TILE, min((tx + 1) * TILE, W))
    ys = np.arange(ty * TILE, min((ty + 1) * TILE, H))
    gy, gx = np.meshgrid(ys, xs, indexing="ij")
    return gx.ravel(), gy.ravel()


def tile_candidates(pr: Projected, order: np.ndarray, tx: int, ty: int) -> np.ndarray:
    """Visible primitives (in depth order) whose tile rect contains tile (tx, ty)."""
    r = pr.rect[order]
    m = (r[:, 0] <= tx) & (tx < r[:, 2]) & (r[:, 1] <= ty) & (ty < r[:, 3])
    return order[m]


def render(p: Dict[str, torch.Tensor], cam: Dict[str, object], mode: str = "binned",
           tiles: Optional[Sequence[tuple]] = None, scene_f32=None, pr: Optional[Projected] = None,
           chunk: int = 4096, attenuation: bool = False, mip2d: bool = False, filter3d=None,
           tau_alpha: float = 1e-4, tau_T: float = 1e-3) -> Image:
    """Render the whole image (or only the listed tiles; other pixels are NaN).
    mode 'brute': every visible primitive at every pixel; 'binned': per-tile
    candidate lists from the tile rects (exact culling: the rect covers every
    pixel where o G >= 1/255).  tau_alpha / tau_T: relative width of the
    bands around the alpha and stop thresholds inside which a decision is
    reported fragile (blend_pixels); they change no rendered value."""
    if pr is None:
        pr = project(p, cam, scene_f32, attenuation, mip2d, filter3d)
    W, H = cam["W"], cam["H"]
    bg = cam["bg"]
    order = depth_order(pr.depth32, pr.visible.numpy())
    tx_n, ty_n = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    color = torch.full((H * W, 3), float("nan"), dtype=DT)
    fT = torch.full((H * W,), float("nan"), dtype=DT)
    last = np.full(H * W, -2, np.int64)
    nbl = np.zeros(H * W, np.int64)
    frag = np.zeros(H * W, bool)
    nfrag = np.zeros(H * W, np.int64)
    fbound = np.zeros(H * W)
    if tiles is None:
        tiles = [(tx, ty) for ty in range(ty_n) for tx in range(tx_n)]
    parts = []
    if mode == "brute":
        xs, ys = [], []
        for (tx, ty) in tiles:
            gx, gy = _tile_pixels(tx, ty, W, H)
            xs.append(gx); ys.append(gy)
        gx, gy = np.concatenate(xs), np.concatenate(ys)
        for s in range(0, len(gx), chunk):
            parts.append((gx[s:s + chunk], gy[s:s + chunk], order))
    else:
        for (tx, ty) in tiles:
            gx, gy = _tile_pixels(tx, ty, W, H)
            parts.append((gx, gy, tile_candidates(pr, order, tx, ty)))
    cols, fts, idxs, fms = [], [], [], []
    for gx, gy, cand in parts:
        res = blend_pixels(pr, cand, torch.from_numpy(gx + 0.5).to(DT),
                           torch.from_numpy(gy + 0.5).to(DT), bg, tau_alpha=tau_alpha, tau_T=tau_T)
        idx = gy * W + gx
        cols.append(res.color); fts.append(res.final_T); idxs.append(torch.from_numpy(idx)); fms.append(res.freq_map)
        last[idx] = res.last_id
        nbl[idx] = res.n_blended
        frag[idx] = res.fragile
        nfrag[idx] = res.n_fragile
        fbound[idx] = res.fragile_bound
    fm = torch.full((H * W,), float("nan"), dtype=DT)
    if idxs:
        ii = torch.cat(idxs)
        color = color.index_put((ii,), torch.cat(cols))
        fT = fT.index_put((ii,), torch.cat(fts))
        fm = fm.index_put((ii,), torch.cat(fms))
    vis_t = pr.visible
    span = float((pr.rgb.detach()[vis_t] - bg[None, :]).abs().max()) if bool(vis_t.any()) else 0.0
    return Image(color.T.reshape(3, H, W), fT.reshape(H, W), last.reshape(H, W),
                 nbl.reshape(H, W), frag.reshape(H, W), fm.reshape(H, W), nfrag.reshape(H, W), span,
                 fbound.reshape(H, W))


def render_scene(scene, cam, mode="binned", tiles=None, attenuation=False, mip2d=False, filter3d=None,
                 tau_alpha: float = 1e-4, tau_T: float = 1e-3) -> Image:
    """Convenience: numpy scene/camera objects -> fp64 image."""
    with torch.no_grad():
        return render(scene_tensors(scene), camera_tensors(cam), mode, tiles, scene_f32=scene,
                      attenuation=attenuation, mip2d=mip2d, filter3d=filter3d, tau_alpha=tau_alpha, tau_T=tau_T)


# --------------------------------------------------------------------------
# gradients: exact derivative of the definition above (autograd, fp64)
# --------------------------------------------------------------------------
GRAD_NAMES = ("means", "scales", "quats", "opacities", "colors", "sh", "freqs", "weights")


def render_grads(scene, cam, dl_dimage: np.ndarray, mode="binned", attenuation=False, mip2d=False,
                 filter3d=None) -> Dict[str, np.ndarray]:
    """d(sum dl_dimage * C)/d(params) for every activated attribute (fp64)."""
    p = scene_tensors(scene, requires_grad=True)
    ct = camera_tensors(cam)
    img = render(p, ct, mode, scene_f32=scene, attenuation=attenuation, mip2d=mip2d, filter3d=filter3d)
    g = torch.tensor(np.asarray(dl_dimage, np.float64), dtype=DT)
    (img.color * g).sum().backward()
    # attributes outside the graph (the empty frequency arrays of K = 0) get zeros
    return {k: (v.grad.numpy() if v.grad is not None else np.zeros(tuple(v.shape))) for k, v in p.items()}


def mean2d_grads(scene, cam, dl_dimage: np.ndarray, attenuation=False, mip2d=False, filter3d=None):
    """Per primitive, the gradient of L = sum(dl_dimage * C) with respect to
    its image-plane mean (pixels), two ways: summed over pixels (the
    view-space positional gradient that density control accumulates, Sec.
    3.4.2), and as per-axis sums over pixels of the absolute per-pixel
    gradients |dL_p / d mu2d| (the homodirectional gradient of AbsGS, the
    densification variant that the paper combines with its primitive in Sec.
    4.1 and Table 1).  Every pixel blends with its own copy of the means, so
    autograd hands back each pixel's contribution separately.  Binned mode
    (tile lists from the rects).  Returns (sum [n, 2], abs [n, 2])."""
    ct = camera_tensors(cam)
    with torch.no_grad():
        pr = project(scene_tensors(scene), ct, scene, attenuation, mip2d, filter3d)
    W, H = ct["W"], ct["H"]
    order = depth_order(pr.depth32, pr.visible.numpy())
    g_img = torch.tensor(np.asarray(dl_dimage, np.float64), dtype=DT)
    tot = np.zeros((scene.n, 2))
    ab = np.zeros((scene.n, 2))
    for ty in range((H + TILE - 1) // TILE):
        for tx in range((W + TILE - 1) // TILE):
            cand = tile_candidates(pr, order, tx, ty)
            if len(cand) == 0:
                continue
            gx, gy = _tile_pixels(tx, ty, W, H)
            mu = pr.mu2d[torch.from_numpy(cand)].detach()[None].expand(len(gx), -1, -1).clone()
            mu.requires_grad_(True)
            res = blend_pixels(pr, cand, torch.from_numpy(gx + 0.5).to(DT), torch.from_numpy(gy + 0.5).to(DT),
                               ct["bg"], mu=mu)
            gsel = g_img[:, torch.from_numpy(gy), torch.from_numpy(gx)].T
            (res.color * gsel).sum().backward()
            gp = mu.grad.numpy()
            np.add.at(tot, cand, gp.sum(0))
            np.add.at(ab, cand, np.abs(gp).sum(0))
    return tot, ab


def mip_filter3d(means: np.ndarray, cams: Sequence, s: float = 0.2, margin: float = 0.15):
    """Variance of the 3D smoothing filter of every primitive (Mip-Splatting's
    3D filter, used with the Gabor primitive in Sec. 4.1 and Table 1).  The
    sampling rate of a camera at a primitive is its focal length over the
    primitive's depth, max(fx, fy) / z, counted for the cameras whose frustum
    holds the mean (z > near plane, image point inside the image grown by
    ``margin`` of its size on every side); with the largest rate r the filter
    variance is s / r^2.  A primitive that no camera sees gets the largest
    variance of the others (0 if none is seen).  Returns (variances [n],
    fragile [n]: a frustum decision within rounding distance of its bound)."""
    m = np.asarray(means, np.float64)
    n = m.shape[0]
    best = np.zeros(n)
    seen = np.zeros(n, bool)
    fragile = np.zeros(n, bool)
    for cam in cams:
        R = np.asarray(cam.R, np.float64)
        t = np.asarray(cam.t, np.float64)
        pc = m @ R.T + t
        z = pc[:, 2]
        front = z > cam.near
        zs = np.where(front, z, 1.0)
        x = cam.fx * pc[:, 0] / zs + cam.cx
        y = cam.fy * pc[:, 1] / zs + cam.cy
        lo_x, hi_x = -margin * cam.width, (1.0 + margin) * cam.width
        lo_y, hi_y = -margin * cam.height, (1.0 + margin) * cam.height
        inside = front & (x >= lo_x) & (x <= hi_x) & (y >= lo_y) & (y <= hi_y)
        rate = max(cam.fx, cam.fy) / zs
        best = np.where(inside, np.maximum(best, rate), best)
        seen |= inside
        tol = 1e-3 + 1e-5 * np.abs(x)
        tol_y = 1e-3 + 1e-5 * np.abs(y)
        fragile |= np.abs(z - cam.near) <= 1e-5 * max(1.0, abs(cam.near))
        fragile |= front & ((np.abs(x - lo_x) <= tol) | (np.abs(x - hi_x) <= tol)
                            | (np.abs(y - lo_y) <= tol_y) | (np.abs(y - hi_y) <= tol_y))
    var = np.zeros(n)
    var[seen] = s / best[seen] ** 2
    if seen.any() and not seen.all():
        var[~seen] = var[seen].max()
    return var, fragile


def _take(pr: Projected, rows: np.ndarray, local_i: int, one: Projected) -> Projected:
    """Rows ``rows`` of a projection (detached), with row ``local_i`` replaced
    by the differentiable single-primitive projection ``one``."""
    r = torch.from_numpy(rows)

    def pick(full, single):
        f = full.detach()[r].clone()
        return torch.cat([f[:local_i], single, f[local_i + 1:]], 0)
    out = Projected(visible=pr.visible[r], depth32=pr.depth32[rows],
                    mu2d=pick(pr.mu2d, one.mu2d), cov2d_raw=pr.cov2d_raw.detach()[r],
                    conic=pick(pr.conic, one.conic), opac=pick(pr.opac, one.opac),
                    rgb=pick(pr.rgb, one.rgb), f2d=pick(pr.f2d, one.f2d), w=pick(pr.w, one.w),
                    rect=pr.rect[rows], tiles=pr.tiles[rows], fragile_rect=pr.fragile_rect[rows],
                    fragile_prim=pr.fragile_prim[rows])
    out.w_dc = pick(pr.w_dc, one.w_dc)
    return out


def window_setup(pr_all: Projected, order: np.ndarray, i: int):
    """The window of primitive i: the tiles of its rect, each tile's
    candidates (depth order), the rows of the projection they use and the
    position of i among them.  None when i is not visible."""
    if not bool(pr_all.visible[i]):
        return None
    x0, y0, x1, y1 = (int(v) for v in pr_all.rect[i])
    tiles = [(tx, ty) for ty in range(y0, y1) for tx in range(x0, x1)]
    cands = [tile_candidates(pr_all, order, tx, ty) for (tx, ty) in tiles]
    rows = np.unique(np.concatenate(cands + [np.array([i])]))
    return tiles, cands, rows, int(np.searchsorted(rows, i))


def _row(pr: Projected, i: int) -> Projected:
    """Primitive i's record fields of a projection as a one-row projection
    (only the fields _support_pixels reads)."""
    return Projected(visible=pr.visible[i:i + 1], depth32=pr.depth32[i:i + 1], mu2d=pr.mu2d[i:i + 1],
                     cov2d_raw=pr.cov2d_raw[i:i + 1], conic=pr.conic[i:i + 1], opac=pr.opac[i:i + 1],
                     rgb=pr.rgb[i:i + 1], f2d=pr.f2d[i:i + 1], w=pr.w[i:i + 1], rect=pr.rect[i:i + 1],
                     tiles=pr.tiles[i:i + 1], fragile_rect=pr.fragile_rect[i:i + 1],
                     fragile_prim=pr.fragile_prim[i:i + 1])


def _support_pixels(rec_i: Projected, gx: np.ndarray, gy: np.ndarray, margin: float = 2e-4) -> np.ndarray:
    """Pixels of (gx, gy) where primitive i (its one-row projection) may
    reach alpha >= 1/255: o G >= (1/255)(1 - margin).  Since the Gabor factor
    B is at most 1, alpha <= o G; elsewhere i is skipped (zero derivative) and
    none of its skip decisions is fragile."""
    with torch.no_grad():
        mx, my = float(rec_i.mu2d[0, 0]), float(rec_i.mu2d[0, 1])
        a, b, c = (float(v) for v in rec_i.conic[0])
        o = float(rec_i.opac[0])
    dx, dy = gx + 0.5 - mx, gy + 0.5 - my
    q = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy
    with np.errstate(over="ignore"):
        return o * np.exp(-0.5 * q) >= ALPHA_MIN * (1.0 - margin)


def _window_total(scene, ct, g_img: torch.Tensor, pr_all: Projected, win, i: int, pi,
                  support_only: bool = False) -> torch.Tensor:
    """sum(dl_dimage * C) over the pixels of the tiles in primitive i's rect
    (``win`` from window_setup), with primitive i projected from the
    attribute tensors ``pi`` (a one-row scene) and every other primitive as in
    ``pr_all``.  Outside those tiles primitive i is not a candidate (its alpha
    there is below 1/255), so this window holds every pixel that depends on it.
    support_only keeps only the pixels of _support_pixels: the sum then
    differs by terms that do not depend on i (the same gradient), so it is
    only for differentiation at the given attributes."""
    W, H = ct["W"], ct["H"]
    sub = scene.subset(np.array([i]))
    pri = project(pi, ct, sub)
    total = torch.zeros((), dtype=DT)
    if win is None:
        return total
    tiles, cands, rows, local_i = win
    pr = _take(pr_all, rows, local_i, pri)
    for (tx, ty), cand in zip(tiles, cands):
        gx, gy = _tile_pixels(tx, ty, W, H)
        if support_only:
            keep = _support_pixels(pri, gx, gy)
            if not keep.any():
                continue
            gx, gy = gx[keep], gy[keep]
        loc = np.searchsorted(rows, cand)
        res = blend_pixels(pr, loc, torch.from_numpy(gx + 0.5).to(DT), torch.from_numpy(gy + 0.5).to(DT), ct["bg"])
        gsel = g_img[:, torch.from_numpy(gy), torch.from_numpy(gx)].T
        total = total + (res.color * gsel).sum()
    return total


def primitive_grads_windowed(scene, cam, dl_dimage: np.ndarray, prims: Sequence[int],
                             pr_all: Optional[Projected] = None) -> List[Dict[str, np.ndarray]]:
    """Gradients of sum(dl_dimage * C) w.r.t. the attributes of each listed
    primitive, evaluated exactly by re-rendering only the tiles in that
    primitive's rect (outside them its alpha is below 1/255 and it is skipped,
    so no other pixel depends on it), and in them only the pixels its
    envelope reaches (elsewhere its derivative is zero)."""
    ct = camera_tensors(cam)
    with torch.no_grad():
        if pr_all is None:
            pr_all = project(scene_tensors(scene), ct, scene)
    order = depth_order(pr_all.depth32, pr_all.visible.numpy())
    g_img = torch.tensor(np.asarray(dl_dimage, np.float64), dtype=DT)
    out = []
    for i in prims:
        pi = scene_tensors(scene.subset(np.array([i])), requires_grad=True)
        total = _window_total(scene, ct, g_img, pr_all, window_setup(pr_all, order, i), i, pi, support_only=True)
        if total.requires_grad:
            total.backward()
        grads = {}
        for k, v in pi.items():
            grads[k] = (v.grad.numpy()[0] if v.grad is not None else np.zeros(v.shape[1:]))
        out.append(grads)
    return out


def primitive_loss_windowed(scene, cam, dl_dimage: np.ndarray, i: int, attrs: Dict[str, np.ndarray],
                            pr_all: Optional[Projected] = None, win=None) -> float:
    """sum(dl_dimage * C) over primitive i's window (see _window_total) with
    primitive i's attributes set to ``attrs`` (fp64 arrays of one primitive,
    e.g. perturbed for finite differences); the decisions taken on float32
    values (depth key, culls) stay those of the unperturbed primitive.  ``win``
    (from window_setup) may be passed to reuse the candidate lists."""
    ct = camera_tensors(cam)
    with torch.no_grad():
        if pr_all is None:
            pr_all = project(scene_tensors(scene), ct, scene)
        if win is None:
            win = window_setup(pr_all, depth_order(pr_all.depth32, pr_all.visible.numpy()), i)
        g_img = torch.tensor(np.asarray(dl_dimage, np.float64), dtype=DT)
        pi = {k: torch.tensor(np.asarray(v, np.float64)[None], dtype=DT) for k, v in attrs.items()}
        return float(_window_total(scene, ct, g_img, pr_all, win, i, pi))


# --------------------------------------------------------------------------
# gradient slack of fragile decisions
# --------------------------------------------------------------------------
# A skip decision (alpha against 1/255) or a stop decision (T (1 - alpha)
# against 1e-4) taken within rounding of its threshold may go either way in
# float32.  Either outcome is a correct evaluation of the definition, and the
# gradient is piecewise smooth across them, so a float32 rasterizer's gradient
# can differ from the float64 one by the jump between the two branches.  For
# every fragile decision of a pixel, the oracle evaluates that jump exactly:
# the gradient of dl_p . (C_p(other outcome) - C_p) with respect to every
# attribute of every candidate of the pixel.  The slack of a gradient element
# is the sum of the jumps' magnitudes over all fragile decisions (several may
# flip together; their effects add up to first order).
def record_jacobian(scene, cam, prims: Sequence[int], attenuation=False, mip2d=False,
                    filter3d=None) -> Dict[str, Dict[str, np.ndarray]]:
    """Jacobian of the listed primitives' 2D records with respect to their
    activated attributes: J[field][attr] has shape [len(prims), dim(field),
    *attr_shape] (fields RECORD_FIELDS flattened per primitive).  The
    projection is independent per primitive, so one backward per record
    component over the sum across primitives gives every row."""
    prims = np.asarray(prims, np.int64)
    ct = camera_tensors(cam) if not isinstance(cam, dict) else cam
    sub = scene.subset(prims)
    p = scene_tensors(sub, requires_grad=True)
    fv = None if filter3d is None else np.asarray(filter3d)[prims]
    pr = project(p, ct, sub, attenuation, mip2d, fv)
    names = list(p.keys())
    n = len(prims)
    out: Dict[str, Dict[str, np.ndarray]] = {}
    for f in RECORD_FIELDS:
        val = getattr(pr, f).reshape(n, -1)
        d = val.shape[1]
        out[f] = {a: np.zeros((n, d) + tuple(p[a].shape[1:])) for a in names}
        for c in range(d):
            gr = torch.autograd.grad(val[:, c].sum(), [p[a] for a in names], retain_graph=True, allow_unused=True)
            for a, g in zip(names, gr):
                if g is not None:
                    out[f][a][:, c] = g.numpy()
    return out


def _decision_jumps(pr: Projected, cand: np.ndarray, gx: np.ndarray, gy: np.ndarray, bg: torch.Tensor,
                    g_pix: torch.Tensor, res: PixelResult) -> Optional[Dict[str, np.ndarray]]:
    """For the fragile decisions of ``res`` (a blend of ``cand`` at the pixel
    centres of (gx, gy); g_pix [P, 3] the loss gradient of those pixels), the
    gradient of dl_p . (C_p(flipped) - C_p) with respect to each candidate's
    2D record, one row per decision: field -> [R, m, dim].  None if there is
    no fragile decision."""
    fa, ft = res.frag_alpha, res.frag_stop
    dec = [(pix, j, 0) for pix, j in zip(*np.nonzero(fa))] + [(pix, j, 1) for pix, j in zip(*np.nonzero(ft))]
    if not dec:
        return None
    R, m = len(dec), len(cand)
    rows = np.array([d[0] for d in dec])
    FA = np.zeros((R, m), bool)
    FS = np.zeros((R, m), bool)
    for r, (_, j, kind) in enumerate(dec):
        (FA if kind == 0 else FS)[r, j] = True
    ci = torch.from_numpy(np.asarray(cand, np.int64))
    rec = {}
    for f in RECORD_FIELDS:
        base = getattr(pr, f).detach()[ci]
        rec[f] = base[None].expand((R,) + tuple(base.shape)).clone().requires_grad_(True)
    X = torch.from_numpy(gx[rows] + 0.5).to(DT)
    Y = torch.from_numpy(gy[rows] + 0.5).to(DT)
    flipped = blend_pixels(pr, cand, X, Y, bg, rec=rec, flip_alpha=FA, flip_stop=FS)
    plain = blend_pixels(pr, cand, X, Y, bg, rec=rec)
    ((flipped.color - plain.color) * g_pix[torch.from_numpy(rows)]).sum().backward()
    # fields outside the graph (the empty frequency arrays of K = 0) get zeros
    return {f: (rec[f].grad if rec[f].grad is not None else torch.zeros_like(rec[f])).reshape(R, m, -1).numpy()
            for f in RECORD_FIELDS}


def _jumps_to_attrs(jumps: Dict[str, np.ndarray], J: Dict[str, Dict[str, np.ndarray]],
                    jrows: np.ndarray) -> Dict[str, np.ndarray]:
    """Per decision row and candidate, the jump in attribute space
    |sum_field jump_2d . J|, summed over the rows: attr -> [m, *attr_shape]
    (candidate c uses Jacobian row jrows[c])."""
    out = {}
    for a in J[RECORD_FIELDS[0]]:
        acc = None
        for f in RECORD_FIELDS:
            Jf = J[f][a][jrows]                                   # [m, d, *attr]
            t = np.einsum("rmd,md...->rm...", jumps[f], Jf)
            acc = t if acc is None else acc + t
        out[a] = np.abs(acc).sum(0)
    return out


def render_grad_slack(scene, cam, dl_dimage: np.ndarray, attenuation=False, mip2d=False,
                      filter3d=None, with_mean2d=False) -> Dict[str, np.ndarray]:
    """Slack of every gradient element of render_grads (binned mode): the
    summed magnitudes of the gradient jumps of every fragile decision in the
    image (zero for a primitive no such decision reaches).  with_mean2d adds
    "mean2d" [n, 2]: the same for the image-plane mean gradient of
    mean2d_grads (it also bounds the change of its per-pixel absolute sums)."""
    ct = camera_tensors(cam)
    with torch.no_grad():
        pr = project(scene_tensors(scene), ct, scene, attenuation, mip2d, filter3d)
    W, H = ct["W"], ct["H"]
    order = depth_order(pr.depth32, pr.visible.numpy())
    g_img = torch.tensor(np.asarray(dl_dimage, np.float64), dtype=DT)
    vis = np.nonzero(pr.visible.numpy())[0]
    J = None
    row_of = np.full(scene.n, -1, np.int64)
    row_of[vis] = np.arange(len(vis))
    slack = {a: np.zeros(tuple(v.shape)) for a, v in scene_tensors(scene).items()}
    if with_mean2d:
        slack["mean2d"] = np.zeros((scene.n, 2))
    for ty in range((H + TILE - 1) // TILE):
        for tx in range((W + TILE - 1) // TILE):
            cand = tile_candidates(pr, order, tx, ty)
            if len(cand) == 0:
                continue
            gx, gy = _tile_pixels(tx, ty, W, H)
            X, Y = torch.from_numpy(gx + 0.5).to(DT), torch.from_numpy(gy + 0.5).to(DT)
            with torch.no_grad():
                res = blend_pixels(pr, cand, X, Y, ct["bg"])
            g_pix = g_img[:, torch.from_numpy(gy), torch.from_numpy(gx)].T
            jumps = _decision_jumps(pr, cand, gx, gy, ct["bg"], g_pix, res)
            if jumps is None:
                continue
            if J is None:
                J = record_jacobian(scene, ct, vis, attenuation, mip2d, filter3d)
            per = _jumps_to_attrs(jumps, J, row_of[cand])
            for a, v in per.items():
                np.add.at(slack[a], cand, v)
            if with_mean2d:
                np.add.at(slack["mean2d"], cand, np.abs(jumps["mu2d"]).sum(0))
    return slack


def primitive_grad_slack_windowed(scene, cam, dl_dimage: np.ndarray, prims: Sequence[int],
                                  pr_all: Optional[Projected] = None) -> List[Dict[str, np.ndarray]]:
    """The slack of primitive_grads_windowed: for each listed primitive, the
    summed jump magnitudes of every fragile decision in the tiles of its rect
    (the only pixels it reaches)."""
    ct = camera_tensors(cam)
    with torch.no_grad():
        if pr_all is None:
            pr_all = project(scene_tensors(scene), ct, scene)
    W, H = ct["W"], ct["H"]
    order = depth_order(pr_all.depth32, pr_all.visible.numpy())
    g_img = torch.tensor(np.asarray(dl_dimage, np.float64), dtype=DT)
    out = []
    for i in prims:
        zero = {a: np.zeros(tuple(v.shape[1:])) for a, v in scene_tensors(scene.subset(np.array([i]))).items()}
        win = window_setup(pr_all, order, i)
        if win is None:
            out.append(zero)
            continue
        J = None
        for (tx, ty), cand in zip(win[0], win[1]):
            gx, gy = _tile_pixels(tx, ty, W, H)
            keep = _support_pixels(_row(pr_all, i), gx, gy)
            if not keep.any():
                continue
            gx, gy = gx[keep], gy[keep]
            X, Y = torch.from_numpy(gx + 0.5).to(DT), torch.from_numpy(gy + 0.5).to(DT)
            with torch.no_grad():
                res = blend_pixels(pr_all, cand, X, Y, ct["bg"])
            g_pix = g_img[:, torch.from_numpy(gy), torch.from_numpy(gx)].T
            jumps = _decision_jumps(pr_all, cand, gx, gy, ct["bg"], g_pix, res)
            if jumps is None:
                continue
            if J is None:
                J = record_jacobian(scene, ct, [i])
            c = int(np.nonzero(np.asarray(cand) == i)[0][0])
            one = {f: v[:, c:c + 1] for f, v in jumps.items()}
            per = _jumps_to_attrs(one, J, np.array([0]))
            for a, v in per.items():
                zero[a] += v[0]
        out.append(zero)
    return out


# --------------------------------------------------------------------------
# photometric loss (Sec. 3.4.1): (1 - lambda) L1 + lambda (1 - SSIM), lambda = 0.2
# --------------------------------------------------------------------------
def gaussian_window(size=11, sigma=1.5) -> torch.Tensor:
    x = torch.arange(size, dtype=DT) - size // 2
    g = torch.exp(-(x * x) / (2 * sigma * sigma))
    return g / g.sum()


def ssim_map(img: torch.Tensor, ref: torch.Tensor, size=11, sigma=1.5) -> torch.Tensor:
    """SSIM index map (Wang et al. 2004) with an 11x11 Gaussian window,
    sigma 1.5, zero-padded 'same' filtering, C1 = 0.01^2, C2 = 0.03^2."""
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    g1 = gaussian_window(size, sigma)
    win = (g1[:, None] * g1[None, :])[None, None].expand(img.shape[0], 1, size, size)
    pad = size // 2
    f = lambda z: torch.nn.functional.conv2d(z[None], win, padding=pad, groups=img.shape[0])[0]  # noqa: E731
    mx, my = f(img), f(ref)
    sxx = f(img * img) - mx * mx
    syy = f(ref * ref) - my * my
    sxy = f(img * ref) - mx * my
    return ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))


def photometric_loss(img: torch.Tensor, ref: torch.Tensor, lam=0.2) -> torch.Tensor:
    l1 = (img - ref).abs().mean()
    return (1.0 - lam) * l1 + lam * (1.0 - ssim_map(img, ref).mean())


def loss_and_grad(img: np.ndarray, ref: np.ndarray, lam=0.2):
    x = torch.tensor(np.asarray(img, np.float64), dtype=DT, requires_grad=True)
    r = torch.tensor(np.asarray(ref, np.float64), dtype=DT)
    L = photometric_loss(x, r, lam)
    L.backward()
    return float(L.detach()), x.grad.numpy()
