"""The differentiation path: rasterize() (torch.autograd.Function over mvgs_forward/mvgs_backward)
followed by fused_loss() (the fused L1 + D-SSIM kernel of Sec. 3 and Sec. 5.1.2) and
loss.backward() gives the leaf parameters the library backward's gradients, and these match the
oracle's double-precision gradients; and the frame each forward makes lives exactly as long as
its backward needs it: released by the backward, at once when no backward can follow, when the
graph is dropped, and a stale frame handle is refused by the C ABI."""
import ctypes as C
import gc

import numpy as np
import pytest
import torch

import oracle
from paper_2506_12727_amd import _lib as L
from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer, fused_loss, rasterize

from gpu_common import compare_grad, grad_flags, needs_gpu, to_np

pytestmark = pytest.mark.gpu

PARAMS = ("means", "scales", "quats", "opacities", "sh")


def _case():
    sc = scenes.make_scene(5000, 3, log_scale_mean=-3.1)
    cams = scenes.make_cameras([(96, 64), (61, 47), (40, 90)])
    return sc, cams


def _leaves(sc):
    g = GaussianTensors.from_scene(sc)
    for n in PARAMS:
        getattr(g, n).requires_grad_(True)
    return g


def test_autograd_gradients_equal_library_backward_and_oracle():
    needs_gpu()
    sc, cams = _case()
    w_l1, w_dssim = 0.8, 0.2
    tile = (16, 16)
    flags = grad_flags(sc, cams, tile)
    masks = [torch.from_numpy((f == 0).astype(np.float32)).cuda()[None] for f in flags]
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams)]
    r = Rasterizer(tile)
    g = _leaves(sc)
    imgs = rasterize(r, cams, g)
    # pixels the oracle flags take no image gradient on either side
    for im, m in zip(imgs, masks):
        im.register_hook(lambda gi, m=m: gi * m)
    loss = fused_loss(r, cams, imgs, tg, w_l1, w_dssim)
    loss.backward()
    torch.cuda.synchronize()
    auto = {n: getattr(g, n).grad.detach().clone() for n in PARAMS}
    # the same step through the library calls directly
    g0 = GaussianTensors.from_scene(sc)
    im0, fr = r.forward(g0, cams)
    loss0, dl = r.loss(cams, im0, tg, w_l1, w_dssim)
    assert torch.equal(torch.cat([i.flatten() for i in im0]), torch.cat([i.detach().flatten() for i in imgs]))
    assert float(loss0.item()) == float(loss.item())
    for t, m in zip(dl, masks):
        t.mul_(m)
    lib = r.backward(g0, fr, dl)
    torch.cuda.synchronize()
    for n in PARAMS:
        # float atomics add in any order: equal up to rounding
        assert torch.allclose(auto[n], lib[n], rtol=1e-5, atol=1e-6 * float(lib[n].abs().max())), n
    ob = oracle.backward(sc, cams, to_np(dl), tile, geom32_mode=False)
    for n in PARAMS:
        compare_grad(n, auto[n].cpu().numpy(), ob[n])
    r.release(fr)
    r.close()


def test_autograd_accumulates_statistics():
    needs_gpu()
    sc, cams = _case()
    r = Rasterizer((16, 16))
    g = _leaves(sc)
    dz = dict(e1=torch.zeros(g.P, device="cuda"), e2=torch.zeros(g.P, device="cuda"),
              count=torch.zeros(g.P, dtype=torch.int32, device="cuda"))
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams)]
    fused_loss(r, cams, rasterize(r, cams, g, densify=dz), tg).backward()
    torch.cuda.synchronize()
    want = np.zeros(g.P, np.int64)
    for v in range(len(cams)):
        want += oracle.geom32(sc, cams, v)["participates"]
    assert np.array_equal(dz["count"].cpu().numpy(), want)
    assert float(dz["e1"].sum()) > 0
    r.close()


def test_frame_lifetime():
    needs_gpu()
    sc, cams = _case()
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams)]
    r = Rasterizer((16, 16))
    g = _leaves(sc)
    fused_loss(r, cams, rasterize(r, cams, g), tg).backward()   # sizes the context's buffers
    # the upload ring takes its slots in turn (4 KiB each at first use): fill all of them so that
    # what is held below is workspace and frames only
    with torch.no_grad():
        for _ in range(16):
            rasterize(r, cams, g)
    torch.cuda.synchronize()
    held = r.memory_held()
    # forwards no backward can follow release their frame at once
    with torch.no_grad():
        for _ in range(4):
            rasterize(r, cams, g)
    g_frozen = GaussianTensors.from_scene(sc)
    for _ in range(3):
        rasterize(r, cams, g_frozen)
    # a graph dropped before its backward releases its frame with it
    for _ in range(3):
        imgs = rasterize(r, cams, g)
        del imgs
        gc.collect()
    assert r.memory_held() == held
    # one backward per forward: a second backward raises instead of reading a reused frame
    loss = fused_loss(r, cams, rasterize(r, cams, g), tg)
    loss.backward(retain_graph=True)
    with pytest.raises(RuntimeError, match="already released"):
        loss.backward()
    assert r.memory_held() == held
    r.close()


def test_stale_frame_handle_is_refused():
    """A frame handle kept past mvgs_frame_release is refused (MVGS_EINVAL) even after its pooled
    frame object was reused by a later forward."""
    needs_gpu()
    sc, cams = _case()
    r = Rasterizer((16, 16))
    g = GaussianTensors.from_scene(sc)
    _, f1 = r.forward(g, cams)
    old = C.c_void_p(f1.handle.value)
    r.release(f1)
    _, f2 = r.forward(g, cams)   # takes the same pooled frame object
    assert (f2.handle.value & ((1 << 48) - 1)) == (old.value & ((1 << 48) - 1))
    assert f2.handle.value != old.value
    lib = r.lib
    V = C.c_int64()
    assert lib.mvgs_frame_info(old, C.byref(V), None, None) == L.MVGS_EINVAL
    assert lib.mvgs_frame_release(r.ctx, old) == L.MVGS_EINVAL
    dl = [torch.zeros((3, c.height, c.width), device="cuda") for c in cams]
    grads = {n: torch.empty_like(getattr(g, n)) for n in PARAMS}
    st = lib.mvgs_backward(r.ctx, None, C.byref(r._gauss(g)), old, L.ptr_array([t.data_ptr() for t in dl]),
                           C.byref(r._grads(grads)), None)
    assert st == L.MVGS_EINVAL
    # the live handle still works, and releasing it twice is refused
    assert lib.mvgs_frame_info(f2.handle, C.byref(V), None, None) == L.MVGS_OK and V.value > 0
    h2 = C.c_void_p(f2.handle.value)
    r.release(f2)
    assert lib.mvgs_frame_release(r.ctx, h2) == L.MVGS_EINVAL
    r.close()


def test_capacity_overflow_raises_in_autograd():
    needs_gpu()
    sc, cams = _case()
    r = Rasterizer((16, 16), capacity=(16, 16))
    g = _leaves(sc)
    with pytest.raises(L.MvgsError):
        rasterize(r, cams, g)
    r.close()
