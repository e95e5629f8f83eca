"""mvgs_loss_noalloc, the loss entry point for callers that cannot allocate device memory: through
the C ABI it gives mvgs_loss's loss and dL/dI bit for bit, on two calls in a row (the second on a
smaller batch, over the scratch the first left behind), with L1 and with L1 + D-SSIM, and neither
the context nor PyTorch's allocator holds more memory afterwards."""
import numpy as np
import pytest
import torch

from paper_2506_12727_amd import _lib as L
from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.raster import Rasterizer

from gpu_common import needs_gpu

pytestmark = pytest.mark.gpu


def _batch(sizes, seed):
    cams = scenes.make_cameras(sizes, seed=seed)
    rng = np.random.default_rng(seed)
    imgs = [torch.from_numpy(rng.random((3, c.height, c.width), dtype=np.float32)).cuda() for c in cams]
    tgts = [torch.from_numpy(rng.random((3, c.height, c.width), dtype=np.float32)).cuda() for c in cams]
    return cams, imgs, tgts


def _call(fn, r, cams, imgs, tgts, w_l1, w_dssim, out, grads):
    return fn(r.ctx, None, L.camera_array(cams), len(cams), L.ptr_array([t.data_ptr() for t in imgs]),
              L.ptr_array([t.data_ptr() for t in tgts]), float(w_l1), float(w_dssim), out.data_ptr(),
              L.ptr_array([t.data_ptr() for t in grads]))


# (first batch, second smaller batch, w_l1, w_dssim)
CASES = [([(1920, 1080), (1280, 720), (980, 545)], [(640, 480), (33, 17)], 1.0, 0.0),
         ([(1600, 1064), (320, 240), (161, 97)], [(200, 120)], 0.8, 0.2)]


@pytest.mark.parametrize("first,second,w_l1,w_dssim", CASES)
def test_noalloc_loss_equals_loss(first, second, w_l1, w_dssim):
    needs_gpu()
    lib = L.lib()
    r = Rasterizer((16, 16))
    for k, sizes in enumerate((first, second)):
        cams, imgs, tgts = _batch(sizes, seed=40 + k)
        want_out = torch.empty(1, device="cuda")
        want_g = [torch.full_like(t, float("nan")) for t in imgs]
        assert _call(lib.mvgs_loss, r, cams, imgs, tgts, w_l1, w_dssim, want_out, want_g) == L.MVGS_OK
        out = torch.full((1,), float("nan"), device="cuda")
        grads = [torch.full_like(t, float("nan")) for t in imgs]
        torch.cuda.synchronize()
        held, allocated = r.memory_held(), torch.cuda.memory_allocated()
        st = _call(lib.mvgs_loss_noalloc, r, cams, imgs, tgts, w_l1, w_dssim, out, grads)
        assert st == L.MVGS_OK, lib.mvgs_last_error(r.ctx)
        torch.cuda.synchronize()
        assert r.memory_held() == held and torch.cuda.memory_allocated() == allocated
        assert torch.equal(out, want_out), (k, float(out), float(want_out))
        for a, b in zip(grads, want_g):
            assert torch.equal(a, b), k
    r.close()


def test_noalloc_loss_refuses_what_its_scratch_cannot_hold():
    needs_gpu()
    lib = L.lib()
    r = Rasterizer((16, 16))
    cams, imgs, tgts = _batch([(8, 8)] * 65, seed=7)   # one view more than the kernel-argument table
    out = torch.full((1,), 123.0, device="cuda")
    grads = [torch.full_like(t, 5.0) for t in imgs]
    assert _call(lib.mvgs_loss_noalloc, r, cams, imgs, tgts, 0.8, 0.2, out, grads) == L.MVGS_ECAPACITY
    torch.cuda.synchronize()
    assert float(out) == 123.0 and all(bool((g == 5.0).all()) for g in grads)   # nothing was enqueued
    # 64 of them fit, and a full-HD view with D-SSIM fits too
    for sizes in ([(8, 8)] * 64, [(1920, 1080)]):
        cams, imgs, tgts = _batch(sizes, seed=8)
        out = torch.empty(1, device="cuda")
        grads = [torch.empty_like(t) for t in imgs]
        assert _call(lib.mvgs_loss_noalloc, r, cams, imgs, tgts, 0.8, 0.2, out, grads) == L.MVGS_OK
        want_out, want_g = r.loss(cams, imgs, tgts, 0.8, 0.2)
        torch.cuda.synchronize()
        assert torch.equal(out, want_out) and all(torch.equal(a, b) for a, b in zip(grads, want_g))
    r.close()
