"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/gabsplat.h, and rejects invalid arguments
before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2508_05343_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2508_05343_amd import build
        build.build()
    return _lib


def declared_functions():
    src = open(os.path.join(ROOT, "include", "gabsplat.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gabsplat_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_function_is_exported(L):
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_helpers(L):
    assert L.gabsplat_abi_version() == 7
    assert L.gabsplat_record_floats(0) == 12 and L.gabsplat_record_floats(2) == 20
    assert L.gabsplat_record_floats(4) == 24 and L.gabsplat_record_floats(8) == 36
    assert L.gabsplat_record_floats(9) == -1
    # rows of whole 128-byte lines: quaternion, 3k frequencies, k weights
    assert L.gabsplat_row_floats(0) == 32 and L.gabsplat_row_floats(4) == 32 and L.gabsplat_row_floats(7) == 32
    assert L.gabsplat_row_floats(8) == 64 and L.gabsplat_row_floats(9) == -1 and L.gabsplat_row_floats(-1) == -1
    assert L.gabsplat_grad2d_floats(4) == 24 and L.gabsplat_grad2d_floats(2) == 16
    # the AbsGS columns follow the record's fields
    assert L.gabsplat_grad2d_stride(4, 0) == 24 and L.gabsplat_grad2d_stride(4, L.GRAD_ABS_MEAN2D) == 24
    assert L.gabsplat_grad2d_stride(2, L.GRAD_ABS_MEAN2D) == 20 and L.gabsplat_grad2d_stride(0, 1) == 12
    assert L.gabsplat_grad2d_stride(2, 2) == -1 and L.gabsplat_grad2d_stride(9, 0) == -1
    assert L.gabsplat_mip_filter3d_workspace_size(1000, 3) >= 3 * 80 + 4 * 4
    assert L.gabsplat_mip_filter3d_workspace_size(10, 0) == 0
    assert L.gabsplat_views_bytes(1, 1) > 0
    small = L.gabsplat_bin_sort_workspace_size(1000, 10000, 64)
    big = L.gabsplat_bin_sort_workspace_size(10 ** 6, 2 * 10 ** 7, 4346)
    assert 0 < small < big
    assert L.gabsplat_bin_sort_workspace_size(-1, 10, 10) == 0
    assert L.gabsplat_loss_workspace_size(3, 840, 1297) >= 3 * 3 * 840 * 1297 * 4
    for s in range(6):
        assert L.lib().gabsplat_status_string(s)


def test_invalid_arguments_are_rejected_on_the_host(L):
    lib = L.lib()
    g = L.Geom()
    cam = L.Camera()
    cam.width, cam.height, cam.fx, cam.fy = 16, 16, 10.0, 10.0
    sc = L.Scene()
    sc.n, sc.k = 10, 9  # k above the limit
    st = lib.gabsplat_preprocess(ctypes.byref(sc), 1, None, ctypes.byref(cam), 1, ctypes.byref(g), None)
    assert st == L.INVALID_ARGUMENT
    sc.k = 2  # NULL attribute pointers with n > 0
    st = lib.gabsplat_preprocess(ctypes.byref(sc), 1, None, ctypes.byref(cam), 1, ctypes.byref(g), None)
    assert st == L.INVALID_ARGUMENT
    st = lib.gabsplat_preprocess(None, 1, None, ctypes.byref(cam), 1, ctypes.byref(g), None)
    assert st == L.INVALID_ARGUMENT
    bad = L.Camera()  # zero-sized image
    st = lib.gabsplat_render_fwd(ctypes.byref(g), None, None, ctypes.byref(bad), 1, None, None, None, None, None,
                                 None, None)
    assert st == L.INVALID_ARGUMENT
    st = lib.gabsplat_bin_sort(ctypes.byref(g), ctypes.byref(cam), 1, 10, None, 0, None, None, 10, None, None,
                               None, None)
    assert st == L.INVALID_ARGUMENT
    st = lib.gabsplat_loss_l1_dssim(None, None, 3, 4, 4, 0.2, None, None, None, 0, None)
    assert st == L.INVALID_ARGUMENT
    st = lib.gabsplat_loss_l1_dssim_noalloc(None, None, 3, 4, 4, 0.2, None, None, None)
    assert st == L.INVALID_ARGUMENT
    # beyond the static scratch: refused before any device work (the
    # pointers are never dereferenced)
    fake = 256
    assert lib.gabsplat_loss_workspace_size(3, 1440, 2560) > L.LOSS_NOALLOC_SCRATCH_BYTES
    st = lib.gabsplat_loss_l1_dssim_noalloc(fake, fake, 3, 1440, 2560, 0.2, fake, fake, None)
    assert st == L.SCRATCH_LIMIT
    assert b"static scratch" in lib.gabsplat_status_string(st)
    assert lib.gabsplat_read_overflow(None, None) == L.INVALID_ARGUMENT
    # backward stages other than blend, project or both (checked before any
    # pointer is dereferenced on the device)
    gg = L.Geom()
    gg.views = gg.rec = gg.tiles = fake
    gr = L.SceneGrads()
    gr.grad2d = fake
    for stages in (0, 4, 7, -1):
        st = lib.gabsplat_render_bwd_stages(ctypes.byref(sc), 1, None, ctypes.byref(cam), 1, ctypes.byref(gg), fake,
                                            fake, fake, fake, fake, ctypes.byref(gr), None, stages, None)
        assert st == L.INVALID_ARGUMENT, stages
    # 3D filter flag without variances
    sc.flags = L.FLAG_MIP_3D
    st = lib.gabsplat_preprocess(ctypes.byref(sc), 1, None, ctypes.byref(cam), 1, ctypes.byref(g), None)
    assert st == L.INVALID_ARGUMENT
    st = lib.gabsplat_mip_filter3d(None, 10, ctypes.byref(cam), 1, 0.2, 0.15, None, None, 0, None)
    assert st == L.INVALID_ARGUMENT
    # packed rows: NULL or misaligned destination, invalid scene; a
    # misaligned rows pointer in a scene; scenes of one call that disagree on
    # having rows (all checked before any device work)
    sc.flags = 0
    ok = L.Scene()
    ok.n, ok.k, ok.sh_degree = 10, 2, 0
    ok.means = ok.scales = ok.quats = ok.opacities = ok.sh = ok.freqs = ok.weights = fake
    assert lib.gabsplat_pack_rows(ctypes.byref(ok), None, None) == L.INVALID_ARGUMENT
    assert lib.gabsplat_pack_rows(ctypes.byref(ok), fake + 4, None) == L.INVALID_ARGUMENT
    assert lib.gabsplat_pack_rows(ctypes.byref(sc), fake, None) == L.INVALID_ARGUMENT
    assert lib.gabsplat_pack_rows(None, fake, None) == L.INVALID_ARGUMENT
    g.views = fake
    ok.rows = fake + 8
    st = lib.gabsplat_preprocess(ctypes.byref(ok), 1, None, ctypes.byref(cam), 1, ctypes.byref(g), None)
    assert st == L.INVALID_ARGUMENT
    two = (L.Scene * 2)(ok, ok)
    two[0].rows, two[1].rows = fake, None
    cams2 = (L.Camera * 2)(cam, cam)
    sv = (ctypes.c_int32 * 2)(0, 1)
    st = lib.gabsplat_preprocess(two, 2, sv, cams2, 2, ctypes.byref(g), None)
    assert st == L.INVALID_ARGUMENT
    g.views = None
    # AbsGS statistic requested without its output
    g.views = g.tiles = 1
    st = lib.gabsplat_densify_stats(ctypes.byref(g), ctypes.byref(cam), 1, 10, 1, L.GRAD_ABS_MEAN2D, 1, None, 1, None)
    assert st == L.INVALID_ARGUMENT


def test_missing_library_fails_loudly(L, monkeypatch):
    monkeypatch.setattr(L, "_LIB", None)
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libgabsplat.so")
    with pytest.raises(L.GabsplatError):
        L.lib()


def test_device_scene_requires_colour_rows():
    """Colour coefficients are one row per primitive: a planar [D*3, n] SH
    tensor (or [3, n] colours) is refused instead of being misread.  Correctly
    shaped host tensors pass every check but the last one (device memory)."""
    import torch
    from paper_2508_05343_amd.rasterize import DeviceScene
    n, k = 10, 2
    z = lambda *s: torch.zeros(*s)
    for kw in (dict(sh=z(n, 48), sh_degree=3), dict(colors=z(n, 3))):
        with pytest.raises(ValueError, match="device tensor"):
            DeviceScene(z(3, n), z(3, n), z(4, n), z(n), z(3 * k, n), z(k, n), **kw)
    with pytest.raises(ValueError, match="shape"):
        DeviceScene(z(3, n), z(3, n), z(4, n), z(n), z(3 * k, n), z(k, n), sh=z(48, n), sh_degree=3)
    with pytest.raises(ValueError, match="shape"):
        DeviceScene(z(3, n), z(3, n), z(4, n), z(n), z(3 * k, n), z(k, n), colors=z(3, n))


def test_device_scene_rejects_bad_layouts():
    """Every attribute is checked for dtype, exact shape and contiguity before
    a raw pointer is taken: a transposed view, a short array, a float64 array
    or a mismatched filter array is refused with a ValueError (the kernels
    would otherwise misread it or read past its end)."""
    import torch
    from paper_2508_05343_amd.rasterize import DeviceScene
    n, k = 12, 3
    z = lambda *s: torch.zeros(*s)  # noqa: E731
    good = dict(means=z(3, n), scales=z(3, n), quats=z(4, n), opacities=z(n), freqs=z(3 * k, n), weights=z(k, n))

    def make(**over):
        a = dict(good, **over)
        col = a.pop("colors", z(n, 3))
        return DeviceScene(a["means"], a["scales"], a["quats"], a["opacities"], a["freqs"], a["weights"], colors=col,
                           filter3d=a.get("filter3d"))
    with pytest.raises(ValueError, match="device tensor"):
        make()
    bad = {
        "means": z(n, 3).t(),                    # transposed view: right shape, wrong layout
        "scales": z(3, n - 1),                   # short
        "quats": z(3, n),                        # a missing component
        "opacities": torch.zeros(n, dtype=torch.float64),  # wrong dtype
        "freqs": z(3 * k - 1, n),                # fewer than 3K rows
        "weights": z(k, n + 1)[:, :n],           # strided view
        "colors": z(3, n),                       # planar colours
        "filter3d": z(n + 1),                    # wrong length
    }
    for name, t in bad.items():
        with pytest.raises(ValueError, match="float32|shape|contiguous|weights|means") as ei:
            make(**{name: t})
        assert "device tensor" not in str(ei.value), name
    with pytest.raises(ValueError, match="at most 8"):
        DeviceScene(z(3, n), z(3, n), z(4, n), z(n), z(27, n), z(9, n), colors=z(n, 3))
    with pytest.raises(ValueError, match="exactly one"):
        DeviceScene(z(3, n), z(3, n), z(4, n), z(n), z(3 * k, n), z(k, n))


def test_no_launch_without_a_gfx950(L):
    """Arguments that pass every check stop at the device check when the
    current device is not a gfx950 (here: no device), before any launch."""
    lib = L.lib()
    st0 = lib.gabsplat_check_device()
    if st0 == L.OK:
        pytest.skip("a gfx950 is present: the calls below would launch with placeholder pointers")
    assert st0 in (L.HIP_ERROR, L.UNSUPPORTED_DEVICE)
    fake = 256  # never dereferenced: the call returns before any device work
    wsb = lib.gabsplat_loss_workspace_size(3, 4, 4)
    assert lib.gabsplat_loss_l1_dssim(fake, fake, 3, 4, 4, 0.2, fake, fake, fake, wsb, None) == st0
    assert lib.gabsplat_loss_l1_dssim_noalloc(fake, fake, 3, 4, 4, 0.2, fake, fake, None) == st0
    # a scene whose rows pass the checks reaches the device check too, where
    # the same scene with misaligned rows was refused as an invalid argument
    sc = L.Scene()
    sc.n, sc.k, sc.sh_degree = 10, 2, 0
    sc.means = sc.scales = sc.quats = sc.opacities = sc.sh = sc.freqs = sc.weights = fake
    cam = L.Camera()
    cam.width, cam.height, cam.fx, cam.fy = 16, 16, 10.0, 10.0
    g = L.Geom()
    g.k, g.views = 2, fake
    g.rec = g.depth = g.rect = g.tiles = fake
    sc.rows = fake
    assert lib.gabsplat_preprocess(ctypes.byref(sc), 1, None, ctypes.byref(cam), 1, ctypes.byref(g), None) == st0
    assert lib.gabsplat_pack_rows(ctypes.byref(sc), fake, None) == st0
    sc.rows = fake + 8
    st = lib.gabsplat_preprocess(ctypes.byref(sc), 1, None, ctypes.byref(cam), 1, ctypes.byref(g), None)
    assert st == L.INVALID_ARGUMENT
