"""Capacity mode and HIP-graph capture of the training step, through the C ABI.

Capacity mode runs the same kernels with counts read on the device, so its images and binning
equal the eager forward's bit for bit; overflow is reported by mvgs_frame_check and does no harm.
A captured step is replayed several times with eager work and synchronizations in between; every
replay matches the eager step (images bit for bit, gradients within the gradient tolerance), also
after new targets and new camera poses."""
import numpy as np
import pytest
import torch

from paper_2506_12727_amd import _lib as L
from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.graph import CapturedStep
from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer

from gpu_common import compare_grad, needs_gpu

pytestmark = pytest.mark.gpu

SIZES = [(160, 96), (96, 128), (130, 70)]


def _batch(seed=1):
    sc = scenes.make_scene(20000, 3, log_scale_mean=-3.3)
    cams = scenes.make_cameras(SIZES, seed=seed)
    return sc, cams


def _eager_step(r, g, cams, targets, w_l1, w_dssim, densify=None):
    imgs, fr = r.forward(g, cams)
    loss, dl = r.loss(cams, imgs, targets, w_l1, w_dssim)
    grads = r.backward(g, fr, dl, densify=densify)
    torch.cuda.synchronize()
    info = fr.info()
    r.release(fr)
    return imgs, float(loss.item()), grads, info


def test_capacity_mode_matches_eager():
    needs_gpu()
    sc, cams = _batch()
    g = GaussianTensors.from_scene(sc)
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams)]
    eager = Rasterizer((16, 16))
    imgs_e, fe = eager.forward(g, cams)
    info = fe.info()
    ke, ve, re_ = eager.export_binning(fe)
    cap = Rasterizer((16, 16), capacity=(info["records"] + 999, info["pairs"] + 4999))
    for _ in range(2):   # the second call reuses the buffers sized by the first
        imgs_c, fc = cap.forward(g, cams)
        fc.check()
        ic = fc.info()
        # the depth sort of a capacity-mode forward orders the context's key window (all 32 bits
        # until a check has seen the keys), the eager one only the bits in which this call's keys
        # differ: more passes, the same order
        assert ic.pop("depth_passes") >= info["depth_passes"]
        assert ic == {k: v for k, v in info.items() if k != "depth_passes"}
        for a, b in zip(imgs_c, imgs_e):
            assert torch.equal(a, b)
        kc, vc, rc = cap.export_binning(fc)
        assert torch.equal(kc, ke) and torch.equal(vc, ve) and torch.equal(rc, re_)
        dz = dict(e1=torch.zeros(g.P, device="cuda"), e2=torch.zeros(g.P, device="cuda"),
                  count=torch.zeros(g.P, dtype=torch.int32, device="cuda"))
        dze = {k: torch.zeros_like(v) for k, v in dz.items()}
        _, dlc = cap.loss(cams, imgs_c, tg, 1.0, 0.0)
        gc = cap.backward(g, fc, dlc, densify=dz)
        _, dle = eager.loss(cams, imgs_e, tg, 1.0, 0.0)
        ge = eager.backward(g, fe, dle, densify=dze)
        torch.cuda.synchronize()
        for n in ge:
            compare_grad(n, gc[n].cpu().numpy(), ge[n].cpu().numpy().astype(np.float64), rtol=1e-4, inf=1e-5,
                         l2=1e-4)
        assert torch.equal(dz["count"], dze["count"])
        cap.release(fc)
    # a smaller batch on the same capacity context
    imgs_s, fs = cap.forward(g, cams[1:])
    fs.check()
    for a, b in zip(imgs_s, imgs_e[1:]):
        assert torch.equal(a, b)
    cap.release(fs)
    eager.release(fe)


def test_capacity_mode_matches_eager_above_16_bit_tile_ids():
    """131,072 tiles (two 2048 x 2048 views at 8x8): 32-bit pair keys in both modes."""
    needs_gpu()
    sc = scenes.make_scene(3000, 0, log_scale_mean=-3.2)
    cams = [scenes.make_camera(2048, 2048, (0.0, 0.3, -2.5)), scenes.make_camera(2048, 2048, (0.4, -0.2, -2.7))]
    g = GaussianTensors.from_scene(sc)
    eager = Rasterizer((8, 8))
    imgs_e, fe = eager.forward(g, cams)
    info = fe.info()
    assert info["tiles"] == 131072
    ke, ve, re_ = eager.export_binning(fe)
    cap = Rasterizer((8, 8), capacity=(info["records"] + 999, info["pairs"] + 4999))
    imgs_c, fc = cap.forward(g, cams)
    fc.check()
    for a, b in zip(imgs_c, imgs_e):
        assert torch.equal(a, b)
    kc, vc, rc = cap.export_binning(fc)
    assert torch.equal(kc, ke) and torch.equal(vc, ve) and torch.equal(rc, re_)
    cap.release(fc)
    eager.release(fe)


def test_capacity_overflow_is_reported_and_harmless():
    needs_gpu()
    sc, cams = _batch()
    g = GaussianTensors.from_scene(sc)
    for c in cams:
        c.bg = np.array([0.1, 0.2, 0.3], np.float32)
    eager = Rasterizer((16, 16))
    _, fe = eager.forward(g, cams)
    info = fe.info()
    eager.release(fe)
    for capacity in [(info["records"] // 2, info["pairs"] * 2), (info["records"] * 2, info["pairs"] // 3)]:
        r = Rasterizer((16, 16), capacity=capacity)
        imgs, fr = r.forward(g, cams)
        with pytest.raises(L.MvgsError) as ei:
            fr.check()
        assert ei.value.status == L.MVGS_ECAPACITY
        bg = torch.tensor([0.1, 0.2, 0.3], device="cuda")[:, None, None]
        for im in imgs:
            assert torch.equal(im, bg.expand_as(im))
        dl = [torch.ones_like(im) for im in imgs]
        grads = r.backward(g, fr, dl)
        torch.cuda.synchronize()
        assert all(float(t.abs().max()) == 0.0 for t in grads.values())
        r.release(fr)
        # a batch that fits works on the same context afterwards
        one, f1 = r.forward(g, cams[2:])
        f1.check()
        ref, fe1 = eager.forward(g, cams[2:])
        assert torch.equal(one[0], ref[0])
        r.release(f1)
        eager.release(fe1)
        r.close()


def test_captured_step_replays_match_eager():
    needs_gpu()
    sc, cams = _batch()
    g = GaussianTensors.from_scene(sc)
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams)]
    dz = dict(e1=torch.zeros(g.P, device="cuda"), e2=torch.zeros(g.P, device="cuda"),
              count=torch.zeros(g.P, dtype=torch.int32, device="cuda"))
    step = CapturedStep(g, cams, tg, 0.8, 0.2, tile=(16, 16), densify=dz)
    eager = Rasterizer((16, 16))
    dze = {k: torch.zeros_like(v) for k, v in dz.items()}
    imgs_e, loss_e, grads_e, info = _eager_step(eager, g, cams, tg, 0.8, 0.2, densify=dze)
    # the capture's warm-up call added its statistics once
    base_count = dz["count"].clone()
    other = Rasterizer((8, 8))
    for rep in range(3):
        step.replay()
        torch.cuda.synchronize()
        step.check()
        for a, b in zip(step.images, imgs_e):
            assert torch.equal(a, b)
        assert abs(float(step.loss.item()) - loss_e) <= 1e-6 * abs(loss_e)
        for n in grads_e:
            compare_grad(n, step.grads[n].cpu().numpy(), grads_e[n].cpu().numpy().astype(np.float64), rtol=1e-4,
                         inf=1e-5, l2=1e-4)
        assert torch.equal(dz["count"], base_count + (rep + 1) * dze["count"])
        # eager work of the program between replays
        im, fo = other.forward(g, cams[:2])
        other.release(fo)
        _ = torch.randn(1000, device="cuda").sum().item()
        torch.cuda.synchronize()
    # new targets, written into the graph's tensors
    tg2 = [torch.rand_like(t) for t in tg]
    for dst, src in zip(step.targets, tg2):
        dst.copy_(src)
    step.replay()
    torch.cuda.synchronize()
    _, loss2, grads2, _ = _eager_step(eager, g, cams, tg2, 0.8, 0.2)
    assert abs(float(step.loss.item()) - loss2) <= 1e-6 * abs(loss2)
    compare_grad("means", step.grads["means"].cpu().numpy(), grads2["means"].cpu().numpy().astype(np.float64),
                 rtol=1e-4, inf=1e-5, l2=1e-4)
    # new camera poses of the same sizes
    cams3 = scenes.make_cameras(SIZES, seed=7)
    step.set_cameras(cams3)
    step.replay()
    torch.cuda.synchronize()
    step.check()
    imgs3, loss3, grads3, _ = _eager_step(eager, g, cams3, tg2, 0.8, 0.2)
    for a, b in zip(step.images, imgs3):
        assert torch.equal(a, b)
    assert abs(float(step.loss.item()) - loss3) <= 1e-6 * abs(loss3)
    for n in grads3:
        compare_grad(n, step.grads[n].cpu().numpy(), grads3[n].cpu().numpy().astype(np.float64), rtol=1e-4,
                     inf=1e-5, l2=1e-4)
    # a size change is refused
    with pytest.raises(L.MvgsError):
        step.set_cameras(scenes.make_cameras([(161, 96), (96, 128), (130, 70)]))
    step.close()
    other.close()
    eager.close()


def test_depth_sort_window_is_checked():
    """In capacity mode the depth sort orders the window of depth keys mvgs_frame_check saw last
    (whole 8-bit passes around them); a replay whose keys leave it does nothing and is reported,
    and a step captured again fits the new keys and matches the eager step."""
    needs_gpu()
    sc, cams = _batch()
    g = GaussianTensors.from_scene(sc)
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams)]
    step = CapturedStep(g, cams, tg, 1.0, 0.0, tile=(16, 16))
    far = scenes.make_cameras(SIZES, seed=2, radius=9.0)   # depths around 9: outside the window
    step.set_cameras(far)
    step.replay()
    torch.cuda.synchronize()
    with pytest.raises(L.MvgsError) as ei:
        step.check()
    assert ei.value.status == L.MVGS_ERETRY and "window" in str(ei.value)
    assert all(float(t.abs().max()) == 0.0 for t in step.grads.values())
    step.close()
    step = CapturedStep(g, far, tg, 1.0, 0.0, tile=(16, 16))
    step.replay()
    torch.cuda.synchronize()
    step.check()
    eager = Rasterizer((16, 16))
    imgs_e, loss_e, grads_e, _ = _eager_step(eager, g, far, tg, 1.0, 0.0)
    for a, b in zip(step.images, imgs_e):
        assert torch.equal(a, b)
    for n in grads_e:
        compare_grad(n, step.grads[n].cpu().numpy(), grads_e[n].cpu().numpy().astype(np.float64), rtol=1e-4,
                     inf=1e-5, l2=1e-4)
    step.close()
    eager.close()
