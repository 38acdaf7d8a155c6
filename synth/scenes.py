"""Seeded scene, camera and request generators.

All draws use ``numpy.random.Generator(PCG64(seed))`` in a fixed order
(means -> log-scales -> quaternions -> opacity -> colour/SH -> frequencies ->
weights), so every consumer that asks for the same configuration receives the
same float32 arrays.  Attributes are produced already *activated*: scales are
positive (exp of the drawn log-scale), opacities lie in (0, 1) (logistic of a
normal draw) and frequency weights are non-negative.

Workload shapes follow the paper's setting (Sec. 4, implementation details:
trained scenes of millions of primitives, F frequency terms per primitive,
spherical-harmonic colour of degree 3, Mip-NeRF360 outdoor frames at quarter
resolution such as 1297x840, object-centric orbits at 800x800).  The public
datasets themselves are not available; these synthetic scenes stand in for
them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclass
class Scene:
    """A set of 3D Gabor primitives, AoS float32 arrays, activated values.

    means [n,3]; scales [n,3] (>0); quats [n,4] as (w,x,y,z), unnormalised;
    opacities [n] in (0,1); exactly one of colors [n,3] / sh [n,D,3] is set,
    D = (degree+1)^2; freqs [n,K,3] in cycles per world unit; weights [n,K] >= 0.
    """

    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray
    freqs: np.ndarray
    weights: np.ndarray
    colors: Optional[np.ndarray] = None
    sh: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def k(self) -> int:
        return int(self.weights.shape[1])

    @property
    def sh_degree(self) -> int:
        if self.sh is None:
            return -1
        return int(round(math.sqrt(self.sh.shape[1]))) - 1

    def subset(self, idx: np.ndarray) -> "Scene":
        return Scene(
            means=self.means[idx].copy(),
            scales=self.scales[idx].copy(),
            quats=self.quats[idx].copy(),
            opacities=self.opacities[idx].copy(),
            freqs=self.freqs[idx].copy(),
            weights=self.weights[idx].copy(),
            colors=None if self.colors is None else self.colors[idx].copy(),
            sh=None if self.sh is None else self.sh[idx].copy(),
            meta=dict(self.meta),
        )

    def nbytes(self) -> int:
        tot = 0
        for a in (self.means, self.scales, self.quats, self.opacities, self.freqs,
                  self.weights, self.colors, self.sh):
            if a is not None:
                tot += a.nbytes
        return tot


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    A world point x maps to camera space as R @ x + t.  ``eye`` is the camera
    centre in world space (kept explicitly for the view direction of the
    spherical-harmonic colour).  Pixel (px, py) samples the image point
    (px + 0.5, py + 0.5).
    """

    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray  # [3,3] float32
    t: np.ndarray  # [3] float32
    eye: np.ndarray  # [3] float32
    near: float = 0.2
    bg: Tuple[float, float, float] = (0.0, 0.0, 0.0)

    @property
    def tiles_x(self) -> int:
        return (self.width + 15) // 16

    @property
    def tiles_y(self) -> int:
        return (self.height + 15) // 16

    @property
    def num_tiles(self) -> int:
        return self.tiles_x * self.tiles_y

    @property
    def num_pixels(self) -> int:
        return self.width * self.height


def look_at(eye, target, down=(0.0, 1.0, 0.0)):
    """World-to-camera rotation/translation for a camera at ``eye`` looking at
    ``target``; ``down`` is the world direction that should map to image +y."""
    eye = np.asarray(eye, np.float64)
    target = np.asarray(target, np.float64)
    z = target - eye
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(down, np.float64), z)
    nx = np.linalg.norm(x)
    if nx < 1e-8:  # looking straight along the down axis: pick another hint
        x = np.cross(np.array([0.0, 0.0, 1.0]), z)
        nx = np.linalg.norm(x)
    x /= nx
    y = np.cross(z, x)
    R = np.stack([x, y, z], 0)
    t = -R @ eye
    return R, t


def pinhole_camera(width, height, hfov_deg, eye, target, down=(0.0, 1.0, 0.0),
                   near=0.2, bg=(0.0, 0.0, 0.0)) -> Camera:
    fx = (width / 2.0) / math.tan(math.radians(hfov_deg) / 2.0)
    R, t = look_at(eye, target, down)
    return Camera(width=int(width), height=int(height), fx=float(np.float32(fx)),
                  fy=float(np.float32(fx)), cx=float(np.float32(width / 2.0)),
                  cy=float(np.float32(height / 2.0)), R=R.astype(np.float32),
                  t=t.astype(np.float32), eye=np.asarray(eye, np.float32),
                  near=float(near), bg=tuple(float(b) for b in bg))


# --------------------------------------------------------------------------
# primitive attribute draws
# --------------------------------------------------------------------------
def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def _attributes(rng, n, k, sh_degree, log_scale_mu, log_scale_sigma,
                freq_sigma=4.0, dc_mu=0.5, sh_sigma=0.2):
    """Draw everything after the means, in the fixed order."""
    log_s = rng.normal(log_scale_mu, log_scale_sigma, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    quats /= np.linalg.norm(quats, axis=1, keepdims=True)
    opac = _sigmoid(rng.normal(0.0, 1.0, size=n))
    colors = sh = None
    if sh_degree < 0:
        colors = rng.uniform(0.0, 1.0, size=(n, 3))
    else:
        d = (sh_degree + 1) ** 2
        sh = np.empty((n, d, 3))
        sh[:, 0, :] = rng.normal(dc_mu, sh_sigma, size=(n, 3))
        if d > 1:
            sh[:, 1:, :] = rng.normal(0.0, sh_sigma, size=(n, d - 1, 3))
    freqs = rng.normal(0.0, freq_sigma, size=(n, k, 3))
    w = rng.uniform(0.0, 1.0, size=(n, k))
    if k > 0:
        w /= np.maximum(1.0, w.sum(axis=1, keepdims=True))
    f32 = lambda a: None if a is None else np.ascontiguousarray(a, np.float32)  # noqa: E731
    return dict(scales=f32(np.exp(log_s)), quats=f32(quats), opacities=f32(opac),
                colors=f32(colors), sh=f32(sh), freqs=f32(freqs), weights=f32(w))


def uniform_scene(seed, n, k, sh_degree=-1, lo=(-1, -1, -1), hi=(1, 1, 1),
                  log_scale_mu=-3.0, log_scale_sigma=0.5, freq_sigma=4.0) -> Scene:
    """Means uniform in a box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    means = rng.uniform(np.asarray(lo, float), np.asarray(hi, float), size=(n, 3))
    attrs = _attributes(rng, n, k, sh_degree, log_scale_mu, log_scale_sigma, freq_sigma)
    return Scene(means=means.astype(np.float32), **attrs, meta=dict(seed=seed))


def ball_scene(seed, n, k, sh_degree=3, radius=1.0, log_scale_mu=-4.0,
               log_scale_sigma=0.7) -> Scene:
    """Means uniform in a ball (object-centric multi-view workload)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.uniform(0.0, 1.0, size=n) ** (1.0 / 3.0)
    means = d * r[:, None]
    attrs = _attributes(rng, n, k, sh_degree, log_scale_mu, log_scale_sigma)
    return Scene(means=means.astype(np.float32), **attrs, meta=dict(seed=seed))


def clustered_scene(seed, n, k=4, sh_degree=3, n_clusters=64, centre_box=8.0,
                    box=10.0, log_scale_mu=-4.0, log_scale_sigma=0.7) -> Scene:
    """Means from a mixture of anisotropic Gaussian clusters inside a
    2*box-unit cube (samples outside are redrawn)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(-centre_box, centre_box, size=(n_clusters, 3))
    stds = rng.uniform(0.5, 2.5, size=(n_clusters, 3))
    rots = _random_orthonormal(rng, n_clusters)
    wts = rng.uniform(0.5, 1.5, size=n_clusters)
    wts /= wts.sum()
    assign = rng.choice(n_clusters, size=n, p=wts)
    means = np.empty((n, 3))
    todo = np.arange(n)
    while todo.size:
        z = rng.normal(size=(todo.size, 3)) * stds[assign[todo]]
        pts = np.einsum("nij,nj->ni", rots[assign[todo]], z) + centres[assign[todo]]
        means[todo] = pts
        bad = np.any(np.abs(pts) > box, axis=1)
        todo = todo[bad]
    attrs = _attributes(rng, n, k, sh_degree, log_scale_mu, log_scale_sigma)
    return Scene(means=means.astype(np.float32), **attrs,
                 meta=dict(seed=seed, centres=centres.astype(np.float32)))


def _random_orthonormal(rng, m):
    """m random 3x3 orthonormal matrices (QR of Gaussian matrices)."""
    a = rng.normal(size=(m, 3, 3))
    qm, rm = np.linalg.qr(a)
    return qm * np.sign(np.diagonal(rm, axis1=1, axis2=2))[:, None, :]


# --------------------------------------------------------------------------
# the named workloads
# --------------------------------------------------------------------------
def scene_1k_k2_rgb(seed=1001) -> Scene:
    """1,000 primitives, K=2, RGB colour, means U[-1,1]^3, log-scales N(-3,0.5)."""
    return uniform_scene(seed, 1000, 2, sh_degree=-1)


def camera_128() -> Camera:
    """128x128, 60 degree horizontal FOV, at distance 3 looking at the origin."""
    return pinhole_camera(128, 128, 60.0, eye=(0.0, 0.0, -3.0), target=(0.0, 0.0, 0.0))


def scene_1m_k4_sh3(seed=1002, n=1_000_000) -> Scene:
    """1M primitives, K=4, SH degree 3, 64 clusters in a 20-unit box."""
    return clustered_scene(seed, n, k=4, sh_degree=3)


def camera_1297x840() -> Camera:
    """1297x840 pinhole inside the scene at (0,0,-6) looking along +z."""
    return pinhole_camera(1297, 840, 60.0, eye=(0.0, 0.0, -6.0), target=(0.0, 0.0, 0.0))


def scene_300k_k4_sh3(seed=1004, n=300_000) -> Scene:
    """300k primitives, K=4, SH3, means uniform in the unit ball."""
    return ball_scene(seed, n, 4, sh_degree=3)


def orbit_cameras_64x800(n_views=64, res=800, radius=4.0, elev_deg=30.0, hfov=40.0) -> List[Camera]:
    """Orbit of cameras at 30 degree elevation looking at the origin, white bg."""
    cams = []
    el = math.radians(elev_deg)
    for v in range(n_views):
        az = 2.0 * math.pi * v / n_views
        eye = (radius * math.cos(el) * math.cos(az), -radius * math.sin(el),
               radius * math.cos(el) * math.sin(az))
        cams.append(pinhole_camera(res, res, hfov, eye=eye, target=(0.0, 0.0, 0.0),
                                   bg=(1.0, 1.0, 1.0)))
    return cams


SERVING_SCENE_SIZES = (100_000, 250_000, 500_000, 1_000_000, 1_000_000, 1_500_000,
                       2_000_000, 2_000_000)
SERVING_RESOLUTIONS = ((256, 256), (800, 800), (1297, 840), (1920, 1080))


def serving_scenes(sizes: Sequence[int] = SERVING_SCENE_SIZES, base_seed=1005) -> List[Scene]:
    return [clustered_scene(base_seed + 2000 + s, int(n), k=4, sh_degree=3)
            for s, n in enumerate(sizes)]


@dataclass
class Request:
    rid: int
    arrival_s: float
    scene: int
    camera: Camera


def serving_requests(scenes: Sequence[Scene], n_requests=2000, qps=200.0, seed=1005,
                     resolutions=SERVING_RESOLUTIONS) -> List[Request]:
    """Poisson arrivals; scene uniform; resolution uniform; random camera in the
    box looking at a random cluster centre of the chosen scene."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / qps, size=n_requests)
    arr = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n_requests):
        s = int(rng.integers(len(scenes)))
        w, h = resolutions[int(rng.integers(len(resolutions)))]
        eye = rng.uniform(-6.0, 6.0, size=3)
        cen = scenes[s].meta.get("centres")
        tgt = cen[int(rng.integers(len(cen)))] if cen is not None else np.zeros(3)
        if np.linalg.norm(tgt - eye) < 1e-3:
            tgt = tgt + np.array([0.0, 0.0, 1.0])
        reqs.append(Request(i, float(arr[i]), s, pinhole_camera(w, h, 60.0, eye, tgt)))
    return reqs


# --------------------------------------------------------------------------
# stage-level synthetic inputs
# --------------------------------------------------------------------------
def random_geom(seed, n, tiles_x, tiles_y, p_visible=0.8, max_extent=6, tie_frac=0.2):
    """Random per-primitive tile rectangles and positive fp32 depths for the
    binning/sorting stage.  Returns (rect [n,4] int32 as x0,y0,x1,y1 exclusive
    upper bounds, depth [n] float32, visible [n] bool).  A share of depths is
    drawn from a tiny set so that equal keys occur."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vis = rng.uniform(size=n) < p_visible
    x0 = rng.integers(0, tiles_x, size=n)
    y0 = rng.integers(0, tiles_y, size=n)
    ex = rng.integers(1, max_extent + 1, size=n)
    ey = rng.integers(1, max_extent + 1, size=n)
    x1 = np.minimum(x0 + ex, tiles_x)
    y1 = np.minimum(y0 + ey, tiles_y)
    depth = rng.uniform(0.2, 50.0, size=n).astype(np.float32)
    ties = rng.uniform(size=n) < tie_frac
    depth[ties] = rng.choice(np.array([1.0, 2.5, 7.25], np.float32), size=int(ties.sum()))
    rect = np.stack([x0, y0, x1, y1], 1).astype(np.int32)
    rect[~vis] = 0
    return rect, depth, vis


def random_dl_dimage(seed, shape, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return (scale * rng.normal(size=shape)).astype(np.float32)


def random_target(seed, shape):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=shape).astype(np.float32)
