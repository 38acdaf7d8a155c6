"""Pins of the oracle's plug-in variants: Mip-Splatting's 3D smoothing filter
and 2D filter on the Gabor primitive's envelope, the per-camera sampling-rate
filter variance, and the AbsGS homodirectional mean gradient with its split
rule (Sec. 4.1 and Table 1 combine the Gabor primitive with both).

Each check is against something other than the oracle's own formula: a
numerical convolution, a hand-computed closed form, finite differences of
the forward, or a plain decision loop."""
import math

import numpy as np
import torch

import synth
from oracle import density_oracle as D
from oracle import gabor_oracle as O


def _scene(means, scales, quats, opac, colors, freqs, weights):
    return synth.Scene(means=np.asarray(means, np.float32), scales=np.asarray(scales, np.float32),
                       quats=np.asarray(quats, np.float32), opacities=np.asarray(opac, np.float32),
                       colors=np.asarray(colors, np.float32), sh=None,
                       freqs=np.asarray(freqs, np.float32), weights=np.asarray(weights, np.float32))


def _axis_camera(W=32, H=32, f=40.0, t=(0.0, 0.0, 0.0), fy=None):
    return synth.Camera(width=W, height=H, fx=f, fy=f if fy is None else fy, cx=W / 2, cy=H / 2,
                        R=np.eye(3, dtype=np.float32), t=np.asarray(t, np.float32),
                        eye=-np.asarray(t, np.float32), bg=(0.0, 0.0, 0.0))


def test_3d_filter_is_the_convolution_with_an_isotropic_gaussian():
    """o' exp(-x^T Sigma'^-1 x / 2) from the filtered envelope equals the
    numerical 3D convolution of o exp(-x^T Sigma^-1 x / 2) with the normalised
    Gaussian of variance v."""
    s = torch.tensor([[0.3, 0.5, 0.2]], dtype=O.DT)
    q = torch.tensor([[0.9, 0.2, -0.3, 0.25]], dtype=O.DT)
    o = torch.tensor([0.7], dtype=O.DT)
    v = 0.04
    s_f, o_f = O.filtered_envelope(s, o, np.array([v]))
    Sig = O.covariance_3d(s, q)[0].numpy()
    Sig_f = O.covariance_3d(s_f, q)[0].numpy()
    h = 0.04
    ax = np.arange(-2.6, 2.6 + h / 2, h)
    Y = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    Si = np.linalg.inv(Sig)
    env = 0.7 * np.exp(-0.5 * np.einsum("ni,ij,nj->n", Y, Si, Y))
    for x0 in ([0.0, 0.0, 0.0], [0.3, -0.2, 0.1], [0.6, 0.4, -0.5]):
        d = np.asarray(x0) - Y
        ker = np.exp(-0.5 * (d * d).sum(1) / v) / (2 * math.pi * v) ** 1.5
        conv = (env * ker).sum() * h ** 3
        x = np.asarray(x0)
        ref = float(o_f[0]) * math.exp(-0.5 * x @ np.linalg.inv(Sig_f) @ x)
        assert abs(conv - ref) <= 1e-9 * ref, (x0, conv, ref)


def test_2d_filter_is_the_convolution_with_the_pixel_gaussian():
    """With the 2D filter, the record's envelope o'' exp(-d^T C d / 2) equals
    the numerical 2D convolution of the undilated footprint o exp(-d^T S^-1 d
    / 2) with the normalised Gaussian of variance 0.1 px^2."""
    cam = _axis_camera()
    sc = _scene([[0.1, -0.05, 2.0]], [[0.05, 0.03, 0.04]], [[0.95, 0.1, 0.2, -0.15]], [0.8],
                [[0.5, 0.5, 0.5]], np.zeros((1, 1, 3)), np.zeros((1, 1)))
    ct = O.camera_tensors(cam)
    pr = O.project(O.scene_tensors(sc), ct, sc, mip2d=True)
    S = pr.cov2d_raw[0].numpy()
    a, b, c = (float(t) for t in pr.conic[0])
    C = np.array([[a, b], [b, c]])
    h = 0.02
    ax = np.arange(-8.0, 8.0 + h / 2, h)
    Y = np.stack(np.meshgrid(ax, ax, indexing="ij"), -1).reshape(-1, 2)
    env = float(sc.opacities[0]) * np.exp(-0.5 * np.einsum("ni,ij,nj->n", Y, np.linalg.inv(S), Y))
    v = 0.1
    for d0 in ([0.0, 0.0], [0.7, -0.4], [-1.5, 1.1]):
        d = np.asarray(d0) - Y
        ker = np.exp(-0.5 * (d * d).sum(1) / v) / (2 * math.pi * v)
        conv = (env * ker).sum() * h * h
        x = np.asarray(d0)
        ref = float(pr.opac[0]) * math.exp(-0.5 * x @ C @ x)
        assert abs(conv - ref) <= 1e-9 * ref, (d0, conv, ref)


def test_3d_filter_reaches_the_projection():
    """An axis-aligned primitive filtered with variance v projects exactly
    like the unfiltered primitive with scales sqrt(s^2 + v) and opacity
    o prod s / sqrt(s^2 + v) (hand-computed)."""
    cam = _axis_camera()
    s = np.array([0.05, 0.08, 0.03])
    v = 0.002
    base = dict(means=[[0.05, 0.0, 2.0]], quats=[[1, 0, 0, 0]], colors=[[0.5, 0.5, 0.5]],
                freqs=[[[1.5, -2.0, 4.0]]], weights=[[0.3]])
    sc = _scene(scales=[s], opac=[0.8], **base)
    s32 = s.astype(np.float32).astype(np.float64)
    sf = np.sqrt(s32 ** 2 + v)
    o2 = float(np.float32(0.8)) * np.prod(s32 / sf)
    ct = O.camera_tensors(cam)
    pa = O.project(O.scene_tensors(sc), ct, sc, filter3d=np.array([v]))
    p = O.scene_tensors(sc)
    p["scales"] = torch.tensor(sf[None], dtype=O.DT)
    p["opacities"] = torch.tensor([o2], dtype=O.DT)
    pb = O.project(p, ct, sc)
    for name in ("mu2d", "conic", "opac", "f2d", "w"):
        np.testing.assert_allclose(getattr(pa, name).numpy(), getattr(pb, name).numpy(), rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(pa.rect, pb.rect)


def test_filter3d_variance_closed_forms():
    f, s = 40.0, 0.2
    near_cam = _axis_camera(f=f)                         # primitive at depth 2
    far_cam = _axis_camera(f=f, t=(0.0, 0.0, 1.0))       # the same primitive at depth 3
    wide = _axis_camera(f=20.0, fy=30.0, t=(0.0, 0.0, 2.0))  # depth 4, sampling rate 30 / 4
    means = np.array([[0.0, 0.0, 2.0],
                      [0.96, 0.0, 2.0],      # x = 1.1 W in near_cam: inside the grown frustum
                      [1.12, 0.0, 2.0],      # x = 1.2 W in near_cam: outside; inside far_cam (x = 30.9 px)
                      [0.0, 0.0, -3.5]])     # behind every camera
    var, frag = O.mip_filter3d(means, [far_cam, near_cam], s)
    assert not frag.any()
    assert math.isclose(var[0], s * (2.0 / f) ** 2, rel_tol=1e-12)
    assert math.isclose(var[1], s * (2.0 / f) ** 2, rel_tol=1e-12)
    assert math.isclose(var[2], s * (3.0 / f) ** 2, rel_tol=1e-12)
    assert math.isclose(var[3], var.max(), rel_tol=0) and var[3] == var[2]
    v1, _ = O.mip_filter3d(means[:1], [wide], s)
    assert math.isclose(v1[0], s * (4.0 / 30.0) ** 2, rel_tol=1e-12)
    v0, _ = O.mip_filter3d(means[3:], [near_cam], s)
    assert v0[0] == 0.0


def _small_scene(seed, n=14, k=2):
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.uniform(2.0, 4.0, n)
    xy = rng.uniform(-0.3, 0.3, (n, 2)) * z[:, None]
    return _scene(np.concatenate([xy, z[:, None]], 1), np.exp(rng.normal(-2.3, 0.3, (n, 3))),
                  rng.normal(size=(n, 4)), rng.uniform(0.3, 0.9, n), rng.uniform(0, 1, (n, 3)),
                  rng.normal(0, 3.0, (n, k, 3)), rng.uniform(0.05, 0.4, (n, k)))


def test_abs_mean_gradient_against_per_pixel_finite_differences():
    """Per primitive and axis: the sum over pixels of the per-pixel mean
    gradient and the sum of its absolute values equal those of central finite
    differences of every pixel's loss term g_p . C_p (means moved by +-h, the
    tile lists kept)."""
    sc = _small_scene(3)
    cam = _axis_camera()
    ct = O.camera_tensors(cam)
    g = synth.random_dl_dimage(4, (3, cam.height, cam.width)).astype(np.float64)
    tot, ab = O.mean2d_grads(sc, cam, g)
    with torch.no_grad():
        pr0 = O.project(O.scene_tensors(sc), ct, sc)
    vis = np.flatnonzero(pr0.visible.numpy())
    assert len(vis) >= 6
    assert np.all(ab >= np.abs(tot) - 1e-15)
    h = 1e-6
    for i in vis[:6]:
        for axis in (0, 1):
            lp = []
            for sgn in (1.0, -1.0):
                pr = O.project(O.scene_tensors(sc), ct, sc)
                mu = pr.mu2d.detach().clone()
                mu[i, axis] += sgn * h
                pr.mu2d = mu
                img = O.render(None, ct, pr=pr)
                lp.append((img.color.detach().numpy() * g).sum(0))
            fd = (lp[0] - lp[1]) / (2 * h)
            assert abs(fd.sum() - tot[i, axis]) <= 1e-6 * max(np.abs(fd).sum(), 1e-12), (i, axis)
            assert abs(np.abs(fd).sum() - ab[i, axis]) <= 1e-6 * max(np.abs(fd).sum(), 1e-12), (i, axis)
    # a primitive whose pixels all pull one way: the two statistics agree
    one = _scene([[0.0, 0.0, 2.0]], [[0.05, 0.05, 0.05]], [[1, 0, 0, 0]], [0.6], [[1.0, 1.0, 1.0]],
                 np.zeros((1, 0, 3)), np.zeros((1, 0)))
    gx = np.zeros((3, cam.height, cam.width))
    gx[:, :, 18:] = 1.0  # only pixels right of the mean carry weight
    t1, a1 = O.mean2d_grads(one, cam, gx)
    assert t1[0, 0] > 0 and math.isclose(a1[0, 0], t1[0, 0], rel_tol=1e-12)  # moving right brightens them
    assert a1[0, 1] > abs(t1[0, 1])  # vertically the pixels pull both ways


def test_abs_statistic_units_and_split_rule():
    acc, den, acc_abs = np.zeros(3), np.zeros(3), np.zeros(3)
    D.accumulate_stats(np.array([[1e-4, 0.0], [0.0, 1e-4], [3e-4, 4e-4]]), np.array([True, True, False]),
                       200, 100, acc, den, np.array([[3e-4, 0.0], [0.0, 2e-4], [1.0, 1.0]]), acc_abs)
    np.testing.assert_allclose(acc_abs, [3e-4 * 100, 2e-4 * 50, 0.0], rtol=1e-12)
    sc = synth.uniform_scene(5, 2000, 2, sh_degree=1, log_scale_mu=-4.6, log_scale_sigma=1.0)
    rng = np.random.Generator(np.random.PCG64(9))
    denom = rng.integers(0, 5, sc.n).astype(np.float32)
    accum = (rng.exponential(0.0002, sc.n) * denom).astype(np.float32)
    accum_abs = (accum * rng.uniform(1.0, 4.0, sc.n)).astype(np.float32)
    prm = D.DensifyParams(abs_grad_threshold=0.0004)
    kind = D.decide(sc, accum, denom, prm, accum_abs)
    for i in range(sc.n):
        avg = np.float32(accum[i] / denom[i]) if denom[i] > 0 else np.float32(0)
        avg_abs = np.float32(accum_abs[i] / denom[i]) if denom[i] > 0 else np.float32(0)
        small = max(sc.scales[i]) <= np.float32(0.01)
        if sc.opacities[i] < np.float32(0.01):
            exp = 3
        elif small:
            exp = 1 if avg >= np.float32(0.0002) else 0
        else:
            exp = 2 if (avg >= np.float32(0.0002) or avg_abs >= np.float32(0.0004)) else 0
        assert kind[i] == exp, i
    plain = D.decide(sc, accum, denom, D.DensifyParams())
    assert ((kind == 2) & (plain == 0)).any()  # the absolute statistic splits more
    assert np.all(kind[plain == 2] == 2)
