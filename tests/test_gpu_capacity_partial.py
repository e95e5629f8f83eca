"""Partial rendering (Alg. 3) in capacity mode and under HIP-graph capture, through the C ABI.

In capacity mode the selection kernels take their task count from the device, so a partial frame
equals the eager one bit for bit (plane, transmittance, depth, merge, 3D loss) and its gradients
agree within the gradient tolerance. A rejected selection, a selection of W*H pixels that is no
partition of the plane, or too small a capacity voids the frame: mvgs_frame_check reports it and
the backward leaves zero gradients. A captured partial step (sub-sampling, forward, merge, 3D
loss, backward) replays with new keys, targets and poses and matches the eager step each time."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2506_12727_amd import _lib as L
from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.graph import CapturedStep, measure_capacity
from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer

from gpu_common import compare_grad, needs_gpu

pytestmark = pytest.mark.gpu

SIZE = (150, 100)   # ragged tiles in both directions at 16 x 16
B = 4


def _setup(seed=3, P=20000):
    sc = scenes.make_scene(P, 3, log_scale_mean=-3.3)
    cams = scenes.make_cameras([SIZE] * B, seed=seed)
    g = GaussianTensors.from_scene(sc)
    tg = [torch.from_numpy(t).cuda() for t in scenes.make_targets(cams)]
    return g, cams, tg


def _keys(seed):
    k = np.random.default_rng(seed).integers(0, 2 ** 32, size=SIZE[0] * SIZE[1], dtype=np.uint64).astype(np.uint32)
    return torch.from_numpy(k.view(np.int32)).cuda()


def _stats(P):
    return dict(e1=torch.zeros(P, device="cuda"), e2=torch.zeros(P, device="cuda"),
                count=torch.zeros(P, dtype=torch.int32, device="cuda"))


def _partial_step(r, g, cams, tg, keys, w_l1=0.8, w_dssim=0.2, densify=None, check=False):
    W, H = SIZE
    off, pix = r.subsample(cams, keys)
    plane = torch.zeros((3, H, W), device="cuda")
    _, fr = r.forward_partial(g, cams, off, pix, L.MVGS_PARTIAL_COMPACT, images=[plane] * len(cams))
    if check:
        fr.check()
    target = r.merge(fr, tg)
    loss, dl = r.loss_3d(fr, plane, target, w_l1, w_dssim)
    grads = r.backward(g, fr, [dl] * len(cams), densify=densify)
    t_fin = [torch.full((H, W), -1.0, device="cuda") for _ in cams]
    r.export_transmittance(fr, t_fin)
    depth = r.export_depth(fr)
    torch.cuda.synchronize()
    r.release(fr)
    return dict(plane=plane, target=target, loss=float(loss.item()), dl=dl, grads=grads, t=t_fin, depth=depth)


def _same_step(a, b):
    assert torch.equal(a["plane"], b["plane"])
    assert torch.equal(a["target"], b["target"])
    assert torch.equal(a["dl"], b["dl"])
    assert a["loss"] == b["loss"]
    for x, y in zip(a["t"], b["t"]):
        assert torch.equal(x, y)
    for x, y in zip(a["depth"], b["depth"]):
        assert torch.equal(x, y)
    for n in a["grads"]:
        compare_grad(n, a["grads"][n].cpu().numpy(), b["grads"][n].cpu().numpy().astype(np.float64), rtol=1e-4,
                     inf=1e-5, l2=1e-4)


@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 16)])
def test_capacity_partial_matches_eager(tile):
    needs_gpu()
    g, cams, tg = _setup()
    cap = Rasterizer(tile, capacity=measure_capacity(g, cams, tile))
    eager = Rasterizer(tile)
    for seed in (1, 2):   # the second call reuses the buffers the first sized
        keys = _keys(seed)
        dz_e, dz_c = _stats(g.P), _stats(g.P)
        e = _partial_step(eager, g, cams, tg, keys, densify=dz_e)
        c = _partial_step(cap, g, cams, tg, keys, densify=dz_c, check=True)
        _same_step(c, e)
        assert torch.equal(dz_c["count"], dz_e["count"])
        assert float(e["plane"].abs().sum()) > 0.0
    # the binary-mask mode on the same capacity context
    keys = _keys(5)
    off, pix = eager.subsample(cams, keys)
    ims_e, fe = eager.forward_partial(g, cams, off, pix, L.MVGS_PARTIAL_MASKED)
    ims_c, fc = cap.forward_partial(g, cams, off, pix, L.MVGS_PARTIAL_MASKED)
    fc.check()
    torch.cuda.synchronize()
    for a, b in zip(ims_c, ims_e):
        assert torch.equal(a, b)
    eager.release(fe)
    cap.release(fc)
    cap.close()
    eager.close()


def test_capacity_partial_void_frames_are_reported():
    needs_gpu()
    g, cams, tg = _setup(P=6000)
    cap_ok = measure_capacity(g, cams)
    r = Rasterizer((16, 16), capacity=cap_ok)
    keys = _keys(7)
    off, pix = r.subsample(cams, keys)
    o = off.cpu().numpy().view(np.uint32).copy()
    p = pix.cpu().numpy().view(np.uint32).copy()
    W, H = SIZE
    assert o[1] > o[0]

    def run(o_, p_, n=None):
        ot = torch.from_numpy(o_.view(np.int32)).cuda()
        pt = torch.from_numpy(p_.view(np.int32)).cuda()
        plane = torch.zeros((3, H, W), device="cuda")
        fr = C.c_void_p()
        st = r.lib.mvgs_forward_partial(r.ctx, None, C.byref(r._gauss(g)), L.camera_array(cams), B, ot.data_ptr(),
                                        pt.data_ptr(), len(p_) if n is None else n, L.MVGS_PARTIAL_COMPACT,
                                        L.ptr_array([plane.data_ptr()] * B), C.byref(fr))
        assert st == 0, r.lib.mvgs_last_error(r.ctx).decode()
        st = r.lib.mvgs_frame_check(r.ctx, None, fr)
        msg = r.lib.mvgs_last_error(r.ctx).decode() if st else ""
        # the backward of a void frame leaves zero gradients
        grads = dict(means=torch.full_like(g.means, 3.0), scales=torch.full_like(g.scales, 3.0),
                     quats=torch.full_like(g.quats, 3.0), opacities=torch.full_like(g.opacities, 3.0),
                     sh=torch.full_like(g.sh, 3.0))
        dl = torch.ones((3, H, W), device="cuda")
        assert r.lib.mvgs_backward(r.ctx, None, C.byref(r._gauss(g)), fr, L.ptr_array([dl.data_ptr()] * B),
                                   C.byref(r._grads(grads)), None) == 0
        torch.cuda.synchronize()
        zero = all(float(t.abs().max()) == 0.0 for t in grads.values())
        r.lib.mvgs_frame_release(r.ctx, fr)
        return st, msg, zero

    st, _, zero = run(o, p)
    assert st == 0 and not zero
    out = p.copy()
    out[o[0]] = W - 1   # the last pixel of row 0 lies in the last tile of the row, not tile 0
    st, msg, zero = run(o, out)
    assert st == L.MVGS_EINVAL and "outside" in msg and zero
    huge = p.copy()
    huge[o[0]] = W * H + 3
    st, msg, zero = run(o, huge)
    assert st == L.MVGS_EINVAL and "outside" in msg and zero
    dup = p.copy()
    dup[o[0] + 1] = dup[o[0]]
    st, msg, zero = run(o, dup)
    assert st == L.MVGS_EINVAL and "twice" in msg and zero
    st, msg, zero = run(o, p, n=len(p) - 1)
    assert st == L.MVGS_EINVAL and "offsets" in msg and zero
    # W*H pixels that are no partition: tile 0 of view 1 takes view 0's pixels of that tile (and
    # as many of its own as it needs to keep its count)
    t1 = (len(o) - 1) // B   # tiles per view; segment t1 is tile 0 of view 1
    seg0, seg1 = p[o[0]:o[1]], p[o[t1]:o[t1 + 1]]
    n0, n1 = len(seg0), len(seg1)
    take = np.sort(np.concatenate([seg0[:n1], seg1[:max(0, n1 - n0)]])).astype(np.uint32)
    assert len(take) == n1 and len(np.unique(take)) == n1
    over = p.copy()
    over[o[t1]:o[t1 + 1]] = take
    st, msg, zero = run(o, over)
    assert st == L.MVGS_EINVAL and "partition" in msg
    # records or pairs over the capacities
    small = Rasterizer((16, 16), capacity=(cap_ok[0] // 3, cap_ok[1]))
    off2, pix2 = small.subsample(cams, keys)
    plane = torch.zeros((3, H, W), device="cuda")
    _, fr = small.forward_partial(g, cams, off2, pix2, L.MVGS_PARTIAL_COMPACT, images=[plane] * B)
    with pytest.raises(L.MvgsError) as ei:
        fr.check()
    assert ei.value.status == L.MVGS_ECAPACITY
    grads = small.backward(g, fr, [torch.ones_like(plane)] * B)
    torch.cuda.synchronize()
    assert all(float(t.abs().max()) == 0.0 for t in grads.values())
    small.release(fr)
    small.close()
    # the context still renders a good selection
    st, _, zero = run(o, p)
    assert st == 0 and not zero
    r.close()


def test_captured_partial_step_replays_match_eager():
    needs_gpu()
    g, cams, tg = _setup(seed=11)
    dz = _stats(g.P)
    step = CapturedStep(g, cams, tg, 0.8, 0.2, tile=(16, 16), densify=dz, partial=True)
    eager = Rasterizer((16, 16))
    other = Rasterizer((8, 8))
    seen = []
    for rep in range(3):
        base = dz["count"].clone()
        step.replay()
        torch.cuda.synchronize()
        step.check()
        keys = step.keys.clone()
        seen.append(keys)
        dze = _stats(g.P)
        e = _partial_step(eager, g, cams, tg, keys, densify=dze)
        assert torch.equal(step.plane, e["plane"])
        assert torch.equal(step.target_plane, e["target"])
        assert float(step.loss.item()) == e["loss"]
        for n in e["grads"]:
            compare_grad(n, step.grads[n].cpu().numpy(), e["grads"][n].cpu().numpy().astype(np.float64), rtol=1e-4,
                         inf=1e-5, l2=1e-4)
        assert torch.equal(dz["count"], base + dze["count"])
        # eager work of the program between replays
        _, fo = other.forward(g, cams[:2])
        other.release(fo)
        _ = torch.randn(1000, device="cuda").sum().item()
        torch.cuda.synchronize()
    # every replay drew new keys
    assert not torch.equal(seen[0], seen[1]) and not torch.equal(seen[1], seen[2])
    # new targets and poses
    tg2 = [torch.rand_like(t) for t in tg]
    for dst, src in zip(step.targets, tg2):
        dst.copy_(src)
    cams3 = scenes.make_cameras([SIZE] * B, seed=29)
    step.set_cameras(cams3)
    step.replay()
    torch.cuda.synchronize()
    step.check()
    e = _partial_step(eager, g, cams3, tg2, step.keys.clone())
    assert torch.equal(step.plane, e["plane"])
    assert float(step.loss.item()) == e["loss"]
    compare_grad("means", step.grads["means"].cpu().numpy(), e["grads"]["means"].cpu().numpy().astype(np.float64),
                 rtol=1e-4, inf=1e-5, l2=1e-4)
    step.close()
    # keys written by the caller
    step2 = CapturedStep(g, cams, tg, 1.0, 0.0, tile=(16, 16), partial=True, fresh_keys=False)
    k = _keys(41)
    step2.keys.copy_(k)
    step2.replay()
    torch.cuda.synchronize()
    step2.check()
    e = _partial_step(eager, g, cams, tg, k, 1.0, 0.0)
    assert torch.equal(step2.plane, e["plane"])
    assert float(step2.loss.item()) == e["loss"]
    step2.close()
    other.close()
    eager.close()
