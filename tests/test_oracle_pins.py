"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

None of these tests re-derives the oracle's formula by retyping it: each one
checks it against a closed form, a numerical integral, a library routine, a
brute-force loop or an invariance the paper states.
"""
import json
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import gabor_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def make_scene(means, scales, quats, opac, colors, freqs=None, weights=None, sh=None):
    n = len(means)
    if freqs is None:
        freqs = np.zeros((n, 0, 3))
        weights = np.zeros((n, 0))
    return synth.Scene(means=np.asarray(means, np.float32), scales=np.asarray(scales, np.float32),
                       quats=np.asarray(quats, np.float32), opacities=np.asarray(opac, np.float32),
                       colors=None if colors is None else np.asarray(colors, np.float32),
                       sh=None if sh is None else np.asarray(sh, np.float32),
                       freqs=np.asarray(freqs, np.float32), weights=np.asarray(weights, np.float32))


def axis_camera(W=32, H=32, f=40.0, bg=(0.0, 0.0, 0.0)):
    """Camera at the origin looking along +z, identity rotation."""
    return synth.Camera(width=W, height=H, fx=f, fy=f, cx=W / 2, cy=H / 2,
                        R=np.eye(3, dtype=np.float32), t=np.zeros(3, np.float32),
                        eye=np.zeros(3, np.float32), bg=bg)


def tiny_scene(seed, n=12, k=2, sh_degree=1):
    """A few primitives in front of an axis camera, sized to cover a 32x32 image."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.uniform(2.0, 4.0, n)
    xy = rng.uniform(-0.3, 0.3, (n, 2)) * z[:, None]
    means = np.concatenate([xy, z[:, None]], 1)
    scales = np.exp(rng.normal(-2.3, 0.3, (n, 3)))
    q = rng.normal(size=(n, 4))
    op = rng.uniform(0.3, 0.9, n)
    sh = rng.normal(0, 0.3, (n, (sh_degree + 1) ** 2, 3)) if sh_degree >= 0 else None
    col = None if sh_degree >= 0 else rng.uniform(0, 1, (n, 3))
    fr = rng.normal(0, 3.0, (n, k, 3))
    w = rng.uniform(0.05, 0.4, (n, k))
    return make_scene(means, scales, q, op, col, fr, w, sh)


# ---------------------------------------------------------------- closed forms
def test_single_axis_aligned_primitive_closed_form():
    """Axis-aligned primitive on the optical axis: the 2D covariance is
    diag((fx sx/tz)^2, (fy sy/tz)^2) + 0.3 I and the 2D frequency is
    (fx_f tz/fx, fy_f tz/fy); one primitive blends as c a + (1 - a) bg."""
    cam = axis_camera(W=32, H=32, f=40.0, bg=(0.2, 0.3, 0.4))
    tz = 2.0
    s = np.array([0.05, 0.08, 0.03])
    f = np.array([1.5, -2.0, 7.0])
    w = 0.35
    sc = make_scene([[0, 0, tz]], [s], [[1, 0, 0, 0]], [0.8], [[0.9, 0.5, 0.1]],
                    [[f]], [[w]])
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    s32 = s.astype(np.float32).astype(np.float64)
    f32 = f.astype(np.float32).astype(np.float64)
    cov = np.diag([(40 * s32[0] / tz) ** 2, (40 * s32[1] / tz) ** 2])
    np.testing.assert_allclose(pr.cov2d_raw[0].numpy(), cov, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(pr.f2d[0, 0].numpy(), [f32[0] * tz / 40, f32[1] * tz / 40], rtol=1e-12)
    img = O.render_scene(sc, cam, "brute")
    for (py, px) in [(16, 16), (15, 17), (18, 12), (16, 20)]:
        dx, dy = px + 0.5 - 16.0, py + 0.5 - 16.0
        G = math.exp(-0.5 * (dx * dx / (cov[0, 0] + 0.3) + dy * dy / (cov[1, 1] + 0.3)))
        w32 = float(np.float32(w))
        B = (1 - w32) + w32 * math.cos(2 * math.pi * (f32[0] * tz / 40 * dx + f32[1] * tz / 40 * dy))
        a = min(0.99, float(np.float32(0.8)) * G * B)
        c = np.array([0.9, 0.5, 0.1], np.float32).astype(np.float64)
        bg = np.array([0.2, 0.3, 0.4])
        exp = c * a + (1 - a) * bg if a >= 1 / 255 else bg
        np.testing.assert_allclose(img.color[:, py, px].numpy(), exp, rtol=1e-12, atol=1e-14)


def test_frequency_along_view_axis_vanishes():
    """A frequency parallel to the viewing direction of an axis-aligned
    primitive integrates out along z: its 2D frequency is zero."""
    cam = axis_camera()
    sc = make_scene([[0, 0, 3.0]], [[0.1, 0.2, 0.3]], [[1, 0, 0, 0]], [0.7], [[1, 1, 1]],
                    [[[0.0, 0.0, 5.0]]], [[0.5]])
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    assert np.abs(pr.f2d.numpy()).max() < 1e-15


def test_two_primitives_closed_form():
    cam = axis_camera(W=16, H=16, f=16.0, bg=(0.1, 0.2, 0.3))
    # both centred on pixel (8, 8): mu2d = (8.5, 8.5)
    sc = make_scene([[1 / 32, 1 / 32, 1.0], [2 / 32, 2 / 32, 2.0]], [[0.05] * 3, [0.1] * 3],
                    [[1, 0, 0, 0]] * 2, [0.6, 0.5], [[1, 0, 0], [0, 0, 1]])
    img = O.render_scene(sc, cam, "brute")
    a1, a2 = float(np.float32(0.6)), float(np.float32(0.5))
    exp = np.array([a1, 0, a2 * (1 - a1)]) + (1 - a1) * (1 - a2) * np.array([0.1, 0.2, 0.3])
    np.testing.assert_allclose(img.color[:, 8, 8].numpy(), exp, rtol=1e-12)
    assert img.n_blended[8, 8] == 2


def test_termination_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "termination_stack.json")))
    W, H = g["width"], g["height"]
    cam = axis_camera(W=W, H=H, f=16.0, bg=tuple(g["bg"]))
    depths = [1.0, 2.0, 3.0, 4.0]
    sc = make_scene([[z / 32, z / 32, z] for z in depths], [[0.05] * 3] * 4, [[1, 0, 0, 0]] * 4,
                    [g["opacity"]] * 4, g["colors"])
    img = O.render_scene(sc, cam, "brute")
    px, py = g["pixel"]
    assert img.n_blended[py, px] == g["expected_n_blended"]
    assert img.last_id[py, px] == 2
    np.testing.assert_allclose(float(img.final_T[py, px]), g["expected_final_T"], rtol=1e-6)
    exp = np.array(g["expected_color"]) + g["expected_final_T"] * np.array(g["bg"])
    np.testing.assert_allclose(img.color[:, py, px].numpy(), exp, rtol=1e-6)
    # the same pixel through the literal sequential loop
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    order = O.depth_order(pr.depth32, pr.visible.numpy())
    c, T, last, cnt = O.blend_pixel_loop(pr, order, px + 0.5, py + 0.5, g["bg"])
    assert cnt == 3 and last == 2
    np.testing.assert_allclose(c, img.color[:, py, px].numpy(), rtol=1e-14)


# ------------------------------------------------- projection vs the paper's form
def _full_jacobian(tc, fx, fy, third):
    tx, ty, tz = tc
    J = np.array([[fx / tz, 0, -fx * tx / tz ** 2], [0, fy / tz, -fy * ty / tz ** 2], third])
    return J


@pytest.mark.parametrize("completion", ["ewa", "unit_z"])
def test_paper_two_step_frequency_formula(completion):
    """f_proj = (JW)^-T f (Sec. 3.3.1) then f2d = f_proj,xy - S_xy,z/S_zz f_proj,z
    with S the inverse of J W Sigma W^T J^T (Sec. 3.3.2), for two different
    completions of J's third row, equals the oracle's 2D frequency."""
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    ct = O.camera_tensors(cam)
    pr = O.project(O.scene_tensors(sc), ct, sc)
    R = cam.R.astype(np.float64)
    checked = 0
    for i in range(0, sc.n, 7):
        m = sc.means[i].astype(np.float64)
        tc = R @ m + cam.t.astype(np.float64)
        u = np.array([cam.fx * tc[0] / tc[2] + cam.cx, cam.fy * tc[1] / tc[2] + cam.cy])
        if not (-0.15 * 128 < u[0] < 1.15 * 128 and -0.15 * 128 < u[1] < 1.15 * 128):
            continue  # guard-band clamp active: J is evaluated elsewhere
        third = tc / np.linalg.norm(tc) if completion == "ewa" else np.array([0.0, 0.0, 1.0])
        A = _full_jacobian(tc, cam.fx, cam.fy, third) @ R
        q = sc.quats[i].astype(np.float64)
        Sig = O.covariance_3d(torch.tensor(sc.scales[i:i + 1].astype(np.float64)),
                              torch.tensor(q[None])).numpy()[0]
        S = np.linalg.inv(A @ Sig @ A.T)
        for k in range(sc.k):
            fp = np.linalg.inv(A).T @ sc.freqs[i, k].astype(np.float64)
            f2 = np.array([fp[0] - S[0, 2] / S[2, 2] * fp[2], fp[1] - S[1, 2] / S[2, 2] * fp[2]])
            np.testing.assert_allclose(pr.f2d[i, k].numpy(), f2, rtol=1e-9, atol=1e-12)
        checked += 1
    assert checked > 50


def test_ray_space_quadrature_of_the_gabor_kernel():
    """Integrating the ray-space 3D Gabor kernel along z numerically gives
    sqrt(2 pi / S_zz) * G2d_raw(d) * exp(-2 pi^2 fz^2 / S_zz) * cos(2 pi f2d . d):
    the oscillating part is exactly cos(2 pi f2d . d) with the oracle's f2d and
    the 2D covariance is the oracle's raw covariance (supplementary A.2, whose
    final formula keeps only the phase; its C2 factor carries the wrong sign)."""
    from scipy.integrate import quad
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    R = cam.R.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(5))
    for i in [3, 50, 222, 777]:
        m = sc.means[i].astype(np.float64)
        tc = R @ m + cam.t.astype(np.float64)
        A = _full_jacobian(tc, cam.fx, cam.fy, tc / np.linalg.norm(tc)) @ R
        Sig = O.covariance_3d(torch.tensor(sc.scales[i:i + 1].astype(np.float64)),
                              torch.tensor(sc.quats[i:i + 1].astype(np.float64))).numpy()[0]
        Spp = A @ Sig @ A.T
        S = np.linalg.inv(Spp)
        fp = np.linalg.inv(A).T @ sc.freqs[i, 0].astype(np.float64)
        sd = math.sqrt(Spp[2, 2])
        for _ in range(3):
            d = rng.normal(0, 1.0, 2) * np.sqrt(np.diag(Spp[:2, :2]))
            def integrand(z):
                x = np.array([d[0], d[1], z])
                return math.exp(-0.5 * x @ S @ x) * math.cos(2 * math.pi * fp @ x)
            val, _ = quad(integrand, -12 * sd, 12 * sd, limit=400, epsabs=1e-14, epsrel=1e-12)
            cov = pr.cov2d_raw[i].numpy()
            f2 = pr.f2d[i, 0].numpy()
            g2 = math.exp(-0.5 * d @ np.linalg.inv(cov) @ d)
            pred = math.sqrt(2 * math.pi / S[2, 2]) * g2 * math.exp(-2 * math.pi ** 2 * fp[2] ** 2 / S[2, 2]) \
                * math.cos(2 * math.pi * f2 @ d)
            assert abs(val - pred) <= 1e-9 * math.sqrt(2 * math.pi / S[2, 2]) + 1e-9 * abs(pred)


def test_covariance_uses_the_perspective_jacobian():
    """The 2D covariance equals J Sigma J^T with J the finite-difference
    Jacobian of the pixel projection t -> (fx tx/tz + cx, fy ty/tz + cy)."""
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    R = cam.R.astype(np.float64)
    proj = lambda t: np.array([cam.fx * t[0] / t[2] + cam.cx, cam.fy * t[1] / t[2] + cam.cy])  # noqa: E731
    for i in range(0, 1000, 97):
        tc = R @ sc.means[i].astype(np.float64) + cam.t.astype(np.float64)
        u = proj(tc)
        if not (0 < u[0] < 128 and 0 < u[1] < 128):
            continue
        h = 1e-6
        Jfd = np.stack([(proj(tc + h * e) - proj(tc - h * e)) / (2 * h) for e in np.eye(3)], 1)
        Sig = O.covariance_3d(torch.tensor(sc.scales[i:i + 1].astype(np.float64)),
                              torch.tensor(sc.quats[i:i + 1].astype(np.float64))).numpy()[0]
        T = Jfd @ R
        np.testing.assert_allclose(pr.cov2d_raw[i].numpy(), T @ Sig @ T.T, rtol=1e-7)
        np.testing.assert_allclose(pr.mu2d[i].numpy(), u, rtol=1e-13)


def test_real_spherical_harmonics_match_scipy():
    """The oracle's real SH basis equals the real combinations of scipy's
    complex spherical harmonics with the Condon-Shortley phase removed."""
    from scipy.special import sph_harm_y
    rng = np.random.Generator(np.random.PCG64(2))
    d = rng.normal(size=(50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = O.sh_basis(torch.tensor(d), 3).numpy()
    theta = np.arccos(d[:, 2])
    phi = np.arctan2(d[:, 1], d[:, 0])
    col = 0
    for l in range(4):
        for m in range(-l, l + 1):
            Yc = sph_harm_y(l, abs(m), theta, phi)
            cs = (-1) ** abs(m)
            if m > 0:
                ref = math.sqrt(2) * cs * Yc.real
            elif m < 0:
                ref = math.sqrt(2) * cs * Yc.imag
            else:
                ref = Yc.real
            np.testing.assert_allclose(Y[:, col], ref, rtol=1e-12, atol=1e-13)
            col += 1


def _rgb(sh, mean, eye):
    return O.sh_to_rgb(torch.tensor(np.asarray(sh, np.float64))[None], torch.tensor(np.asarray(mean, np.float64))[None],
                       torch.tensor(np.asarray(eye, np.float64))).numpy()[0]


# real SH constants of degrees 0-2 (textbook closed forms, no Condon-Shortley phase)
_Y00 = 0.28209479177387814            # 1 / (2 sqrt(pi))
_Y1 = 0.4886025119029199              # sqrt(3 / (4 pi)): y, z, x for m = -1, 0, 1
_Y2A = 1.0925484305920792             # sqrt(15 / pi) / 2: xy, yz, xz
_Y20 = 0.31539156525252005            # sqrt(5 / pi) / 4: 3 z^2 - 1
_Y22 = 0.5462742152960396             # sqrt(15 / pi) / 4: x^2 - y^2


def test_sh_colour_closed_forms():
    """Colour of a primitive from its SH coefficients (Sec. 3.2 keeps the 3DGS
    view-dependent colour): max(0, 0.5 + sum_d c_d Y_d(dir)) with dir the unit
    vector from the camera centre to the mean, coefficients in (l, m) order
    m = -l..l, one coefficient triple (r, g, b) per basis function.  Every
    expected value below is written out by hand from the degree-0..2 closed
    forms: a dropped +0.5, a direction taken from the mean to the camera, a
    permuted basis order or a missing clamp each fails one of them."""
    eye = np.array([0.5, -1.0, 2.0])
    d = np.array([1.0, -2.0, 2.0]) / 3.0           # x = 1/3, y = -2/3, z = 2/3
    mean = eye + 1.5 * 3.0 * d
    # degree 0: a constant plus the offset
    np.testing.assert_allclose(_rgb([[0.4, -0.2, 1.0]], mean, eye),
                               [0.5 + 0.4 * _Y00, 0.5 - 0.2 * _Y00, 0.5 + 1.0 * _Y00], rtol=1e-14)
    # degree 1: Y_1,-1 = c y, Y_1,0 = c z, Y_1,1 = c x; one basis function per channel
    sh1 = [[0.1, 0.1, 0.1], [0.3, 0.0, 0.0], [0.0, 0.3, 0.0], [0.0, 0.0, 0.3]]
    want = [0.5 + 0.1 * _Y00 + 0.3 * _Y1 * (-2.0 / 3.0),
            0.5 + 0.1 * _Y00 + 0.3 * _Y1 * (2.0 / 3.0),
            0.5 + 0.1 * _Y00 + 0.3 * _Y1 * (1.0 / 3.0)]
    np.testing.assert_allclose(_rgb(sh1, mean, eye), want, rtol=1e-14)
    # the reversed direction (camera minus mean) gives a different colour
    flipped = [0.5 + 0.1 * _Y00 - 0.3 * _Y1 * (-2.0 / 3.0), 0.5 + 0.1 * _Y00 - 0.3 * _Y1 * (2.0 / 3.0),
               0.5 + 0.1 * _Y00 - 0.3 * _Y1 * (1.0 / 3.0)]
    assert np.abs(np.asarray(want) - flipped).min() > 0.03
    # the colour depends on the direction only, not on the distance
    np.testing.assert_allclose(_rgb(sh1, eye + 0.01 * d, eye), want, rtol=1e-13)
    # degree 2, one basis function at a time on the red channel
    y2 = [_Y2A * (1 / 3) * (-2 / 3), _Y2A * (-2 / 3) * (2 / 3), _Y20 * (3 * (2 / 3) ** 2 - 1),
          _Y2A * (1 / 3) * (2 / 3), _Y22 * ((1 / 3) ** 2 - (2 / 3) ** 2)]
    for j, yv in enumerate(y2):
        sh2 = np.zeros((9, 3))
        sh2[4 + j, 0] = 1.0
        np.testing.assert_allclose(_rgb(sh2, mean, eye), [0.5 + yv, 0.5, 0.5], rtol=1e-14, err_msg=str(j))
    # clamp at zero, with zero gradient on the clamped channels
    sh0 = torch.tensor([[[-3.0, 0.2, -1.8]]], dtype=torch.float64, requires_grad=True)
    rgb = O.sh_to_rgb(sh0, torch.tensor(mean[None]), torch.tensor(eye))
    np.testing.assert_allclose(rgb.detach().numpy()[0], [0.0, 0.5 + 0.2 * _Y00, 0.0], rtol=1e-14)
    rgb.sum().backward()
    np.testing.assert_allclose(sh0.grad.numpy()[0, 0], [0.0, _Y00, 0.0], rtol=1e-14)


def test_rotation_matrix_is_orthonormal_and_matches_rotation_of_vectors():
    """R(q) v equals the quaternion sandwich q v q* (Hamilton product)."""
    rng = np.random.Generator(np.random.PCG64(3))
    q = rng.normal(size=(20, 4))
    R = O.quat_to_rotmat(torch.tensor(q)).numpy()
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)

    def hprod(a, b):
        w1, x1, y1, z1 = a
        w2, x2, y2, z2 = b
        return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])
    for i in range(20):
        v = rng.normal(size=3)
        conj = qn[i] * np.array([1, -1, -1, -1])
        rv = hprod(hprod(qn[i], np.concatenate([[0], v])), conj)[1:]
        np.testing.assert_allclose(R[i] @ v, rv, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(R[i] @ R[i].T, np.eye(3), atol=1e-12)
        assert np.linalg.det(R[i]) > 0


# ------------------------------------------------------------------ invariants
def _gaussian_splat_loop(pr, order, x, y, bg):
    """Plain 3D Gaussian splatting (Sec. 3.1, Eq. alpha-blend-gauss) at one
    pixel, written independently of the Gabor blend."""
    T, C = 1.0, np.zeros(3)
    for i in order:
        d = np.array([x, y]) - pr.mu2d[i].numpy()
        cov = pr.cov2d_raw[i].numpy() + 0.3 * np.eye(2)
        a = min(0.99, float(pr.opac[i]) * math.exp(-0.5 * d @ np.linalg.solve(cov, d)))
        if a < 1 / 255:
            continue
        if T * (1 - a) < 1e-4:
            break
        C += pr.rgb[i].numpy() * a * T
        T *= 1 - a
    return C + T * np.asarray(bg)


@pytest.mark.parametrize("which", ["weights_zero", "freqs_zero"])
def test_reduces_to_gaussian_splatting(which):
    """With every frequency weight zero, or every frequency zero, the
    primitive is the 3DGS Gaussian (Sec. 3.2.2)."""
    sc = synth.scene_1k_k2_rgb()
    if which == "weights_zero":
        sc.weights[:] = 0
    else:
        sc.freqs[:] = 0
    cam = synth.camera_128()
    img = O.render_scene(sc, cam, "binned")
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    order = O.depth_order(pr.depth32, pr.visible.numpy())
    rng = np.random.Generator(np.random.PCG64(4))
    for _ in range(25):
        px, py = rng.integers(0, 128, 2)
        ref = _gaussian_splat_loop(pr, order, px + 0.5, py + 0.5, cam.bg)
        np.testing.assert_allclose(img.color[:, py, px].numpy(), ref, rtol=1e-10, atol=1e-13)


def test_transmittance_and_convexity():
    """T is in (0, 1]; the colour is a convex combination of the primitive
    colours and the background (weights a_i T_i and T_final sum to one)."""
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    cam.bg = (0.0, 0.0, 0.0)
    img = O.render_scene(sc, cam, "binned")
    T = img.final_T.numpy()
    assert (T > 0).all() and (T <= 1).all()
    # colours are in [0,1] and bg = 0, so every channel is within [0, 1 - T]
    c = img.color.numpy()
    assert (c >= -1e-15).all() and (c <= (1 - T)[None] + 1e-12).all()
    # with all colours = 1 and bg = 1 the image is exactly 1
    sc.colors[:] = 1.0
    cam.bg = (1.0, 1.0, 1.0)
    img = O.render_scene(sc, cam, "binned")
    np.testing.assert_allclose(img.color.numpy(), 1.0, atol=1e-13)


def test_transmittance_monotone_along_the_walk():
    """The final T of ever longer front-to-back candidate prefixes never grows."""
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    order = O.depth_order(pr.depth32, pr.visible.numpy())
    rng = np.random.Generator(np.random.PCG64(6))
    px = torch.tensor(rng.integers(0, 128, 16) + 0.5, dtype=torch.float64)
    py = torch.tensor(rng.integers(0, 128, 16) + 0.5, dtype=torch.float64)
    prev = np.ones(16)
    for j in range(0, len(order) + 1, 10):
        with torch.no_grad():
            T = O.blend_pixels(pr, order[:j], px, py, torch.zeros(3, dtype=torch.float64)).final_T.numpy()
        assert (T <= prev + 1e-15).all() and (T > 0).all()
        prev = T


def test_brute_equals_binned_and_loop():
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    a = O.render_scene(sc, cam, "brute")
    b = O.render_scene(sc, cam, "binned")
    assert float((a.color - b.color).abs().max()) < 1e-14
    assert (a.last_id == b.last_id).all() and (a.n_blended == b.n_blended).all()
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    order = O.depth_order(pr.depth32, pr.visible.numpy())
    rng = np.random.Generator(np.random.PCG64(7))
    for _ in range(20):
        px, py = rng.integers(0, 128, 2)
        c, T, last, cnt = O.blend_pixel_loop(pr, order, px + 0.5, py + 0.5, cam.bg)
        np.testing.assert_allclose(c, a.color[:, py, px].numpy(), rtol=1e-12, atol=1e-14)
        assert last == a.last_id[py, px] and cnt == a.n_blended[py, px]


def test_frequency_sign_and_component_permutation_invariance():
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    base = O.render_scene(sc, cam, "binned")
    s2 = sc.subset(np.arange(sc.n))
    s2.freqs = -s2.freqs
    s2.freqs = s2.freqs[:, ::-1].copy()
    s2.weights = s2.weights[:, ::-1].copy()
    other = O.render_scene(s2, cam, "binned")
    assert float((base.color - other.color).abs().max()) < 1e-13


def test_rigid_motion_invariance():
    """Moving scene (means, orientations, frequency vectors) and camera by the
    same rigid motion leaves the image unchanged: the frequency projection of
    Sec. 3.3.1 transforms covariantly."""
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    base = O.render_scene(sc, cam, "binned")
    rng = np.random.Generator(np.random.PCG64(8))
    qm = rng.normal(size=4)
    qm /= np.linalg.norm(qm)
    Q = O.quat_to_rotmat(torch.tensor(qm[None])).numpy()[0]
    cvec = np.array([0.3, -0.2, 0.5])
    s2 = sc.subset(np.arange(sc.n))
    s2.means = (sc.means.astype(np.float64) @ Q.T + cvec).astype(np.float32)
    w1, x1, y1, z1 = qm
    qs = sc.quats.astype(np.float64)
    w2, x2, y2, z2 = qs.T
    s2.quats = np.stack([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                         w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2],
                        1).astype(np.float32)
    s2.freqs = (sc.freqs.astype(np.float64) @ Q.T).astype(np.float32)
    R2 = cam.R.astype(np.float64) @ Q.T
    t2 = cam.t.astype(np.float64) - R2 @ cvec
    cam2 = synth.Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy, R2.astype(np.float32),
                        t2.astype(np.float32), (Q @ cam.eye.astype(np.float64) + cvec).astype(np.float32))
    other = O.render_scene(s2, cam2, "binned")
    d = (base.color - other.color).abs().numpy()
    ok = ~(base.fragile | other.fragile)
    # fp32 rounding of the moved inputs only
    assert d[:, ok].max() < 2e-4
    assert np.median(d) < 1e-5


# ---------------------------------------------------------------------- sorting
def test_bin_sort_against_brute_force_tuple_sort():
    rect, depth, vis = synth.random_geom(11, 300, 9, 7)
    keys, vals, ranges = O.bin_sort(rect, depth, vis, 9, 63)
    bits = depth.view(np.uint32)
    items = []
    for i in range(300):
        if not vis[i]:
            continue
        for ty in range(rect[i, 1], rect[i, 3]):
            for tx in range(rect[i, 0], rect[i, 2]):
                items.append((ty * 9 + tx, int(bits[i]), i))
    items.sort()
    assert [((t << 32) | b) for t, b, _ in items] == [int(k) for k in keys]
    assert [i for _, _, i in items] == [int(v) for v in vals]
    for t in range(63):
        sel = [p for p, it in enumerate(items) if it[0] == t]
        if sel:
            assert tuple(ranges[t]) == (sel[0], sel[-1] + 1)
        else:
            assert tuple(ranges[t]) == (0, 0)


# --------------------------------------------------------------------- gradients
def _fd_check(scene, cam, g, names, n_elems=6, h=1e-6, seed=0):
    """Central differences of sum(g * C) in fp64 against the autograd gradient."""
    an = O.render_grads(scene, cam, g, mode="brute")
    rng = np.random.Generator(np.random.PCG64(seed))
    worst = 0.0
    for name in names:
        arr = getattr(scene, name)
        for _ in range(n_elems):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            p = O.scene_tensors(scene)
            base = p[name][idx].item()
            vals = []
            for sgn in (+1, -1):
                p2 = {k: v.clone() for k, v in p.items()}
                p2[name][idx] = base + sgn * h * max(1.0, abs(base))
                with torch.no_grad():
                    img = O.render(p2, O.camera_tensors(cam), "brute", scene_f32=scene)
                vals.append(float((img.color.numpy() * g).sum()))
            fd = (vals[0] - vals[1]) / (2 * h * max(1.0, abs(base)))
            a = an[name][idx]
            err = abs(fd - a) / (abs(a) + 1e-6)
            worst = max(worst, err)
            assert abs(fd - a) <= 1e-5 * (abs(a) + 1e-4), (name, idx, fd, a)
    return worst


def test_gradients_match_finite_differences():
    sc = tiny_scene(21)
    cam = axis_camera(bg=(0.3, 0.1, 0.2))
    img = O.render_scene(sc, cam, "brute")
    assert img.fragile.sum() == 0
    g = synth.random_dl_dimage(5, (3, 32, 32))
    _fd_check(sc, cam, g, ["means", "scales", "quats", "opacities", "sh", "freqs", "weights"])


def test_gradients_match_finite_differences_colors_and_guard_band():
    sc = tiny_scene(22, sh_degree=-1)
    sc.means[0] = [1.5, 0.2, 2.0]  # well outside the image: J evaluated at the clamped point
    sc.scales[0] = [0.6, 0.4, 0.5]
    cam = axis_camera(bg=(0.0, 0.5, 1.0))
    g = synth.random_dl_dimage(6, (3, 32, 32))
    _fd_check(sc, cam, g, ["means", "colors", "freqs"], n_elems=8, seed=1)


def test_zero_gradient_invariants():
    """At f = 0 the weights and frequencies get exactly zero gradient; at
    w = 0 the frequencies do (Sec. 3.4.1: a Gabor primitive that degenerates
    to a Gaussian receives no gradient, which is why the paper initialises
    them to small non-zero values)."""
    sc = tiny_scene(23)
    cam = axis_camera()
    g = synth.random_dl_dimage(7, (3, 32, 32))
    s0 = sc.subset(np.arange(sc.n))
    s0.freqs[:] = 0
    gr = O.render_grads(s0, cam, g, "brute")
    scale = np.abs(gr["means"]).max()
    assert scale > 0
    # zero up to the rounding of -g + g summed along two autograd paths
    assert np.abs(gr["weights"]).max() <= 1e-12 * scale and np.abs(gr["freqs"]).max() == 0
    s1 = sc.subset(np.arange(sc.n))
    s1.weights[:] = 0
    gr = O.render_grads(s1, cam, g, "brute")
    assert np.abs(gr["freqs"]).max() == 0
    assert np.abs(gr["weights"]).max() > 0


def test_colour_gradient_closed_form():
    """dC/dc_i = a_i T_i: with g = e_channel at one pixel the colour gradient
    of each primitive is its blend weight."""
    sc = tiny_scene(24, sh_degree=-1)
    cam = axis_camera()
    g = np.zeros((3, 32, 32))
    g[1, 16, 16] = 1.0
    gr = O.render_grads(sc, cam, g, "brute")
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    order = O.depth_order(pr.depth32, pr.visible.numpy())
    T = 1.0
    exp = np.zeros(sc.n)
    for i in order:
        d = np.array([16.5, 16.5]) - pr.mu2d[i].detach().numpy()
        con = pr.conic[i].detach().numpy()
        G = math.exp(-0.5 * (con[0] * d[0] ** 2 + 2 * con[1] * d[0] * d[1] + con[2] * d[1] ** 2))
        Bv = 1 + sum(float(pr.w[i, k]) * (math.cos(2 * math.pi * pr.f2d[i, k].detach().numpy() @ d) - 1)
                     for k in range(sc.k))
        a = min(0.99, float(pr.opac[i]) * G * Bv)
        if a < 1 / 255:
            continue
        if T * (1 - a) < 1e-4:
            break
        exp[i] = a * T
        T *= 1 - a
    np.testing.assert_allclose(gr["colors"][:, 1], exp, rtol=1e-12, atol=1e-15)
    assert np.abs(gr["colors"][:, [0, 2]]).max() == 0


def test_windowed_gradients_equal_full_gradients():
    sc = tiny_scene(25)
    cam = axis_camera()
    g = synth.random_dl_dimage(8, (3, 32, 32))
    full = O.render_grads(sc, cam, g, "binned")
    win = O.primitive_grads_windowed(sc, cam, g, [0, 3, 7])
    for j, i in enumerate([0, 3, 7]):
        for k in ("means", "scales", "quats", "opacities", "sh", "freqs", "weights"):
            np.testing.assert_allclose(win[j][k], full[k][i], rtol=1e-10, atol=1e-14)


# -------------------------------------------------------------------------- loss
def test_ssim_against_brute_force_window_loop():
    rng = np.random.Generator(np.random.PCG64(9))
    x = rng.uniform(size=(3, 9, 10))
    y = rng.uniform(size=(3, 9, 10))
    m = O.ssim_map(torch.tensor(x), torch.tensor(y)).numpy()
    g = np.exp(-((np.arange(11) - 5) ** 2) / (2 * 1.5 ** 2))
    g /= g.sum()
    w2 = np.outer(g, g)
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    for c in range(3):
        for i in range(9):
            for j in range(10):
                acc = np.zeros(5)
                for di in range(-5, 6):
                    for dj in range(-5, 6):
                        ii, jj = i + di, j + dj
                        if 0 <= ii < 9 and 0 <= jj < 10:
                            a, b = x[c, ii, jj], y[c, ii, jj]
                            acc += w2[di + 5, dj + 5] * np.array([a, b, a * a, b * b, a * b])
                mx, my = acc[0], acc[1]
                sxx, syy, sxy = acc[2] - mx * mx, acc[3] - my * my, acc[4] - mx * my
                ref = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx * mx + my * my + C1) * (sxx + syy + C2))
                assert abs(m[c, i, j] - ref) < 1e-12


def test_loss_identity_and_finite_differences():
    rng = np.random.Generator(np.random.PCG64(10))
    x = rng.uniform(size=(3, 12, 14))
    L, g = O.loss_and_grad(x, x)
    assert abs(L) < 1e-15
    y = rng.uniform(size=(3, 12, 14))
    L, g = O.loss_and_grad(x, y)
    for _ in range(10):
        idx = tuple(rng.integers(0, s) for s in x.shape)
        h = 1e-6
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (O.loss_and_grad(xp, y)[0] - O.loss_and_grad(xm, y)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7
    l1 = np.abs(x - y).mean()
    ss = O.ssim_map(torch.tensor(x), torch.tensor(y)).numpy().mean()
    assert abs(L - (0.8 * l1 + 0.2 * (1 - ss))) < 1e-14


# ------------------------------------------------- attenuation-corrected variant
def test_attenuation_closed_form_axis_aligned():
    """Axis-aligned primitive on the optical axis: the z-integration multiplies
    a cosine term by exp(-2 pi^2 f_z^2 s_z^2) (the variance of f . x along the
    ray is f_z^2 s_z^2 there)."""
    cam = axis_camera()
    f = np.array([1.0, -2.0, 3.0])
    s = np.array([0.1, 0.2, 0.15])
    sc = make_scene([[0, 0, 3.0]], [s], [[1, 0, 0, 0]], [0.7], [[1, 1, 1]], [[f]], [[0.5]])
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc, attenuation=True)
    f32, s32 = f.astype(np.float32).astype(float), s.astype(np.float32).astype(float)
    w32 = float(np.float32(0.5))
    np.testing.assert_allclose(float(pr.w[0, 0]), w32 * math.exp(-2 * math.pi ** 2 * (f32[2] * s32[2]) ** 2),
                               rtol=1e-12)
    np.testing.assert_allclose(float(pr.w_dc[0]), 1 - w32, rtol=1e-15)


def test_attenuated_primitive_equals_the_exact_z_integral():
    """With attenuation the 2D Gabor primitive is the exact integral of the
    ray-space 3D primitive along z (supplementary A.2 without dropping the
    per-component factor), up to the common factor sqrt(2 pi / S_zz) that the
    opacity absorbs: checked by fp64 quadrature of the whole filter bank."""
    from scipy.integrate import quad
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc, attenuation=True)
    R = cam.R.astype(np.float64)
    rng = np.random.Generator(np.random.PCG64(12))
    for i in [7, 123, 456, 901]:
        tc = R @ sc.means[i].astype(np.float64) + cam.t.astype(np.float64)
        A = _full_jacobian(tc, cam.fx, cam.fy, tc / np.linalg.norm(tc)) @ R
        Sig = O.covariance_3d(torch.tensor(sc.scales[i:i + 1].astype(np.float64)),
                              torch.tensor(sc.quats[i:i + 1].astype(np.float64))).numpy()[0]
        S = np.linalg.inv(A @ Sig @ A.T)
        fps = [np.linalg.inv(A).T @ sc.freqs[i, k].astype(np.float64) for k in range(sc.k)]
        w = sc.weights[i].astype(np.float64)
        sd = math.sqrt((A @ Sig @ A.T)[2, 2])
        for _ in range(3):
            d = rng.normal(0, 1.0, 2) * np.sqrt(np.diag((A @ Sig @ A.T)[:2, :2]))

            def integrand(z):
                x = np.array([d[0], d[1], z])
                bank = (1 - w.sum()) + sum(w[k] * math.cos(2 * math.pi * fps[k] @ x) for k in range(sc.k))
                return math.exp(-0.5 * x @ S @ x) * bank
            val, _ = quad(integrand, -12 * sd, 12 * sd, limit=400, epsabs=1e-14, epsrel=1e-12)
            g2 = math.exp(-0.5 * d @ np.linalg.inv(pr.cov2d_raw[i].numpy()) @ d)
            bank2 = float(pr.w_dc[i]) + sum(float(pr.w[i, k]) * math.cos(2 * math.pi * pr.f2d[i, k].numpy() @ d)
                                           for k in range(sc.k))
            pred = math.sqrt(2 * math.pi / S[2, 2]) * g2 * bank2
            assert abs(val - pred) <= 1e-9 * math.sqrt(2 * math.pi / S[2, 2])


def test_attenuation_gradients_match_finite_differences():
    sc = tiny_scene(26)
    cam = axis_camera(bg=(0.1, 0.4, 0.2))
    g = synth.random_dl_dimage(13, (3, 32, 32))
    an = O.render_grads(sc, cam, g, mode="brute", attenuation=True)
    rng = np.random.Generator(np.random.PCG64(14))
    for name in ("means", "scales", "quats", "freqs", "weights"):
        arr = getattr(sc, name)
        for _ in range(5):
            idx = tuple(rng.integers(0, s_) for s_ in arr.shape)
            p = O.scene_tensors(sc)
            base = p[name][idx].item()
            h = 1e-6 * max(1.0, abs(base))
            vals = []
            for sgn in (+1, -1):
                p2 = {k: v.clone() for k, v in p.items()}
                p2[name][idx] = base + sgn * h
                with torch.no_grad():
                    img = O.render(p2, O.camera_tensors(cam), "brute", scene_f32=sc, attenuation=True)
                vals.append(float((img.color.numpy() * g).sum()))
            fd = (vals[0] - vals[1]) / (2 * h)
            a = an[name][idx]
            assert abs(fd - a) <= 1e-5 * (abs(a) + 1e-4), (name, idx, fd, a)


def test_frequency_map_is_a_blended_channel():
    """The frequency map equals rendering the scene with every primitive's
    colour set to its weighted frequency sum_k w_k |f2d_k| on a black
    background (same blending weights); for one primitive it is alpha * phi."""
    sc = synth.scene_1k_k2_rgb()
    cam = synth.camera_128()
    img = O.render_scene(sc, cam, "binned")
    pr = O.project(O.scene_tensors(sc), O.camera_tensors(cam), sc)
    phi = (pr.w * torch.linalg.norm(pr.f2d, dim=-1)).sum(-1).numpy()
    s2 = sc.subset(np.arange(sc.n))
    s2.colors = np.repeat(phi[:, None], 3, 1).astype(np.float64)
    with torch.no_grad():
        p2 = O.scene_tensors(s2)
        p2["colors"] = torch.tensor(np.repeat(phi[:, None], 3, 1), dtype=torch.float64)
        ref = O.render(p2, O.camera_tensors(cam), "binned", scene_f32=sc)
    np.testing.assert_allclose(img.freq_map.numpy(), ref.color[0].numpy(), rtol=1e-12, atol=1e-15)
    # one axis-aligned primitive on the axis: alpha * phi at its centre pixel
    one = make_scene([[0, 0, 2.0]], [[0.05, 0.08, 0.03]], [[1, 0, 0, 0]], [0.8], [[1, 1, 1]],
                     [[[1.5, -2.0, 7.0], [0.5, 0.5, 0.0]]], [[0.2, 0.3]])
    c1 = axis_camera(W=32, H=32, f=40.0)
    im1 = O.render_scene(one, c1, "brute")
    f2 = np.array([[1.5, -2.0], [0.5, 0.5]], np.float32).astype(float) * 2.0 / 40.0
    w = np.array([0.2, 0.3], np.float32).astype(float)
    ph = float((w * np.linalg.norm(f2, axis=1)).sum())
    dx = dy = 0.5
    cov = np.diag([(40 * float(np.float32(0.05)) / 2.0) ** 2 + 0.3, (40 * float(np.float32(0.08)) / 2.0) ** 2 + 0.3])
    G = math.exp(-0.5 * (dx * dx / cov[0, 0] + dy * dy / cov[1, 1]))
    B = (1 - w.sum()) + sum(w[k] * math.cos(2 * math.pi * (f2[k, 0] * dx + f2[k, 1] * dy)) for k in range(2))
    a = float(np.float32(0.8)) * G * B
    np.testing.assert_allclose(float(im1.freq_map[16, 16]), a * ph, rtol=1e-12)
