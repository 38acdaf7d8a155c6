"""The allocation-free loss entry point against the workspace one: two calls in
a row through the C ABI (the full 1297x840 training frame, then a smaller
ragged one), each bit for bit equal to gabsplat_loss_l1_dssim on the same
seeded inputs (same kernels, deterministic reduction)."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _pair(seed, shape):
    x = torch.from_numpy(synth.random_target(seed, shape)).cuda()
    y = torch.from_numpy(synth.random_target(seed + 1, shape)).cuda()
    return x, y


def _with_workspace(x, y, lam):
    from paper_2508_05343_amd import _lib
    c, h, w = x.shape
    ws = torch.empty((_lib.gabsplat_loss_workspace_size(c, h, w) + 3) // 4, dtype=torch.float32, device="cuda")
    d_loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grad = torch.empty_like(x)
    _lib.gabsplat_loss_l1_dssim(x, y, lam, d_loss, grad, ws)
    return d_loss, grad


def test_noalloc_loss_equals_workspace_loss_twice(gpu_lib):
    from paper_2508_05343_amd import _lib
    for seed, shape, lam in ((901, (3, 840, 1297), 0.2), (903, (3, 77, 50), 0.35)):
        x, y = _pair(seed, shape)
        ref_loss, ref_grad = _with_workspace(x, y, lam)
        d_loss = torch.full((1,), float("nan"), dtype=torch.float32, device="cuda")
        grad = torch.full_like(x, float("nan"))
        torch.cuda.synchronize()
        _lib.gabsplat_loss_l1_dssim_noalloc(x, y, lam, d_loss, grad)
        torch.cuda.synchronize()
        assert torch.equal(d_loss, ref_loss), (shape, float(d_loss), float(ref_loss))
        assert torch.equal(grad, ref_grad), (shape, float((grad - ref_grad).abs().max()))
        assert np.isfinite(float(d_loss))


def test_noalloc_loss_refuses_beyond_its_scratch(gpu_lib):
    from paper_2508_05343_amd import _lib
    assert _lib.gabsplat_loss_workspace_size(3, 1080, 1920) <= _lib.LOSS_NOALLOC_SCRATCH_BYTES
    big = torch.empty((3, 1440, 2560), dtype=torch.float32, device="cuda")
    assert _lib.gabsplat_loss_workspace_size(3, 1440, 2560) > _lib.LOSS_NOALLOC_SCRATCH_BYTES
    d_loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.GabsplatError, match="static scratch"):
        _lib.gabsplat_loss_l1_dssim_noalloc(big, big, 0.2, d_loss, big)
