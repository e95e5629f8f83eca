"""Partial rendering (Alg. 3) on the GPU, through the C ABI: the sub-sampling equals the oracle's
bit for bit; the thread-efficient and binary-mask modes give, at every selected pixel, the full
forward's value bit for bit (and so the oracle's within the image tolerance) and leave other
pixels alone; their backward equals the oracle's backward of the image gradient restricted to the
selection; bad selections are refused."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
from paper_2506_12727_amd import _lib as L
from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer

from gpu_common import compare_grad, compare_images, needs_gpu, to_np

pytestmark = pytest.mark.gpu

MODES = [L.MVGS_PARTIAL_COMPACT, L.MVGS_PARTIAL_MASKED]
SENTINEL = -7.25


def _keys(W, H, seed):
    k = np.random.default_rng(seed).integers(0, 2 ** 32, size=W * H, dtype=np.uint64).astype(np.uint32)
    return k, torch.from_numpy(k.view(np.int32)).cuda()


def _np(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("tile,B,size", [((16, 16), 4, (61, 47)), ((8, 8), 3, (40, 33)), ((32, 16), 5, (70, 40)),
                                         ((16, 32), 1, (33, 65)), ((8, 8), 70, (8, 8))])
def test_subsample_matches_oracle(tile, B, size):
    needs_gpu()
    W, H = size
    cams = scenes.make_cameras([size] * B)
    kn, kt = _keys(W, H, 3)
    r = Rasterizer(tile)
    off, pix = r.subsample(cams, kt)
    o_off, o_pix = oracle.subsample_tiles(W, H, B, tile, kn)
    assert np.array_equal(_np(off), o_off)
    assert np.array_equal(_np(pix), o_pix)
    r.close()


def _scene_and_sel(tile, B=4, size=(61, 47), seed=9):
    sc = scenes.make_scene(6000, 3, log_scale_mean=-3.0)
    cams = scenes.make_cameras([size] * B)
    kn, kt = _keys(size[0], size[1], seed)
    return sc, cams, kt


def _sel_lists(off, pix, cams, tile):
    """Per view: the selected pixel indices (from the segment layout)."""
    off, pix = _np(off), _np(pix)
    out, base = [], 0
    for c in cams:
        T = ((c.width + tile[0] - 1) // tile[0]) * ((c.height + tile[1] - 1) // tile[1])
        out.append(pix[off[base]:off[base + T]])
        base += T
    return out


@pytest.mark.parametrize("tile,ppl", [((16, 16), 2), ((16, 16), 4), ((32, 16), 4), ((8, 8), 1), ((32, 32), 4)])
@pytest.mark.parametrize("mode", MODES)
def test_partial_forward_equals_full_at_the_selection(tile, ppl, mode):
    needs_gpu()
    sc, cams, kt = _scene_and_sel(tile)
    r = Rasterizer(tile, ppl)
    g = GaussianTensors.from_scene(sc)
    full, ff = r.forward(g, cams)
    off, pix = r.subsample(cams, kt)
    imgs = [torch.full((3, c.height, c.width), SENTINEL, device="cuda") for c in cams]
    imgs, fp = r.forward_partial(g, cams, off, pix, mode, images=imgs)
    merged = torch.full_like(imgs[0], SENTINEL)
    _, fm = r.forward_partial(g, cams, off, pix, mode, images=[merged] * len(cams))
    tf_full = r.export_transmittance(ff)
    tp = [torch.full((c.height, c.width), SENTINEL, device="cuda") for c in cams]
    L.check(r.lib.mvgs_export_transmittance(r.ctx, None, fp.handle, L.ptr_array([t.data_ptr() for t in tp])), r.ctx)
    torch.cuda.synchronize()
    sel = _sel_lists(off, pix, cams, tile)
    covered = np.zeros(cams[0].width * cams[0].height, bool)
    for v, c in enumerate(cams):
        idx = torch.from_numpy(sel[v].astype(np.int64)).cuda()
        a, b = imgs[v].reshape(3, -1), full[v].reshape(3, -1)
        assert torch.equal(a[:, idx], b[:, idx])
        rest = torch.ones(c.width * c.height, dtype=torch.bool, device="cuda")
        rest[idx] = False
        assert bool((a[:, rest] == SENTINEL).all())
        assert torch.equal(merged.reshape(3, -1)[:, idx], b[:, idx])
        assert torch.equal(tp[v].reshape(-1)[idx], tf_full[v].reshape(-1)[idx])
        if mode == L.MVGS_PARTIAL_COMPACT:
            assert bool((tp[v].reshape(-1)[rest] == SENTINEL).all())
        covered[sel[v]] = True
    assert covered.all()   # the views cover the plane: the merged image has no sentinel left
    assert not bool((merged == SENTINEL).any())
    # and the oracle, at the selected pixels of two views
    for v in (0, len(cams) - 1):
        xs, ys = sel[v] % cams[v].width, sel[v] // cams[v].width
        rgb, tf, fl = oracle.render_pixels(sc, cams, v, xs, ys)
        got = imgs[v].cpu().numpy().astype(np.float64)[:, ys, xs].T
        ok = fl == 0
        assert np.all(np.abs(got - rgb)[ok] <= 1e-5 * np.abs(rgb)[ok] + 1e-6)
    for f in (ff, fp, fm):
        r.release(f)
    r.close()


def _uneven_selection(cams, tile, seed):
    """A selection that is not a partition: per (view, tile) a random subset of any size, some
    segments empty, some longer than one wavefront."""
    rng = np.random.default_rng(seed)
    off, pix = [0], []
    for c in cams:
        txn, tyn = (c.width + tile[0] - 1) // tile[0], (c.height + tile[1] - 1) // tile[1]
        for ty in range(tyn):
            for tx in range(txn):
                ps = np.array([y * c.width + x for y in range(ty * tile[1], min(c.height, ty * tile[1] + tile[1]))
                               for x in range(tx * tile[0], min(c.width, tx * tile[0] + tile[0]))])
                k = int(rng.integers(0, len(ps) + 1)) if rng.uniform() > 0.15 else 0
                pick = rng.permutation(ps)[:k]
                pix.extend(pick.tolist())
                off.append(len(pix))
    return (torch.tensor(np.array(off, np.uint32).view(np.int32)).cuda(),
            torch.tensor(np.array(pix, np.uint32).view(np.int32)).cuda())


@pytest.mark.parametrize("mode", MODES)
def test_partial_backward_matches_oracle_on_the_selection(mode):
    needs_gpu()
    tile = (32, 32)
    sc = scenes.make_scene(5000, 3, log_scale_mean=-3.1)
    cams = scenes.make_cameras([(61, 47), (130, 70), (33, 97)])
    r = Rasterizer(tile, 4)
    g = GaussianTensors.from_scene(sc)
    off, pix = _uneven_selection(cams, tile, 12)
    imgs, fp = r.forward_partial(g, cams, off, pix, mode)
    ref = oracle.forward(sc, cams, tile)
    gflags = oracle.forward(sc, cams, tile, geom32_mode=False)["flags"]
    sel = _sel_lists(off, pix, cams, tile)
    rng = np.random.default_rng(13)
    dl_np = []
    for v, c in enumerate(cams):
        d = np.zeros((3, c.height, c.width), np.float32)
        ys, xs = sel[v] // c.width, sel[v] % c.width
        d[:, ys, xs] = rng.normal(size=(3, len(ys))).astype(np.float32) * 1e-3
        d[:, gflags[v] != 0] = 0.0   # pixels whose decisions may differ: on neither side
        dl_np.append(d)
    # the backward reads only selected pixels: garbage elsewhere must not matter
    dl = []
    for v, d in enumerate(dl_np):
        junk = np.full_like(d, 1e3)
        ys, xs = sel[v] // cams[v].width, sel[v] % cams[v].width
        junk[:, ys, xs] = d[:, ys, xs]
        dl.append(torch.from_numpy(junk).cuda())
    dz = dict(e1=torch.zeros(g.P, device="cuda"), e2=torch.zeros(g.P, device="cuda"),
              count=torch.zeros(g.P, dtype=torch.int32, device="cuda"))
    grads = r.backward(g, fp, dl, densify=dz)
    torch.cuda.synchronize()
    ob = oracle.backward(sc, cams, [d.astype(np.float64) for d in dl_np], tile, geom32_mode=False)
    for n in ("means", "scales", "quats", "opacities", "sh"):
        compare_grad(n, grads[n].cpu().numpy(), ob[n])
    compare_grad("e1", dz["e1"].cpu().numpy(), ob["e1"])
    compare_grad("e2", dz["e2"].cpu().numpy(), ob["e2"])
    assert np.array_equal(dz["count"].cpu().numpy(), ob["count"])
    # images at the selection against the oracle's full render
    for v, c in enumerate(cams):
        ys, xs = sel[v] // c.width, sel[v] % c.width
        got = imgs[v].cpu().numpy().astype(np.float64)[:, ys, xs]
        want = ref["images"][v][:, ys, xs]
        ok = ref["flags"][v][ys, xs] == 0
        assert np.all((np.abs(got - want) <= 1e-5 * np.abs(want) + 1e-6)[:, ok])
    r.release(fp)
    r.close()


def test_bad_selections_are_refused():
    needs_gpu()
    tile = (16, 16)
    sc = scenes.make_scene(500, 0)
    cams = scenes.make_cameras([(40, 20), (40, 20)])
    r = Rasterizer(tile)
    g = GaussianTensors.from_scene(sc)
    kn, kt = _keys(40, 20, 1)
    off, pix = r.subsample(cams, kt)
    o, p = _np(off).copy(), _np(pix).copy()

    def run(o_, p_, n=None):
        ot = torch.from_numpy(o_.view(np.int32)).cuda()
        pt = torch.from_numpy(p_.view(np.int32)).cuda()
        fr = C.c_void_p()
        imgs = [torch.zeros((3, 20, 40), device="cuda") for _ in cams]
        st = r.lib.mvgs_forward_partial(r.ctx, None, C.byref(r._gauss(g)), L.camera_array(cams), 2, ot.data_ptr(),
                                        pt.data_ptr(), len(p_) if n is None else n, 0,
                                        L.ptr_array([t.data_ptr() for t in imgs]), C.byref(fr))
        if st == 0:
            r.lib.mvgs_frame_release(r.ctx, fr)
        return st, r.lib.mvgs_last_error(r.ctx).decode()

    assert run(o, p)[0] == 0
    dup = p.copy()
    dup[1] = dup[0]
    st, msg = run(o, dup)
    assert st == L.MVGS_EINVAL and "twice" in msg
    # a repeat in a later round of 64 entries that is itself in ascending order
    assert o[1] - o[0] > 66
    dup2 = p.copy()
    dup2[o[0] + 64] = dup2[o[0] + 63]
    st, msg = run(o, dup2)
    assert st == L.MVGS_EINVAL and "twice" in msg
    out = p.copy()
    out[0] = 39   # pixel (39, 0) lies in tile 2, not tile 0
    st, msg = run(o, out)
    assert st == L.MVGS_EINVAL and "outside" in msg
    bad = o.copy()
    bad[2] = bad[1] - 1
    st, msg = run(bad, p)
    assert st == L.MVGS_EINVAL and "offsets" in msg
    st, msg = run(o, p, n=len(p) - 1)
    assert st == L.MVGS_EINVAL and "offsets" in msg
    huge = p.copy()
    huge[5] = 40 * 20 + 3
    assert run(o, huge)[0] == L.MVGS_EINVAL
    # the context is still usable
    assert run(o, p)[0] == 0
    # sizes that differ cannot be sub-sampled
    with pytest.raises(L.MvgsError):
        r.subsample(scenes.make_cameras([(40, 20), (41, 20)]), kt)
    r.close()


def _merged_setup(tile=(16, 16), B=3, size=(48, 40), seed=21):
    sc = scenes.make_scene(6000, 3, log_scale_mean=-3.0)
    cams = scenes.make_cameras([size] * B, seed=seed)
    kn, kt = _keys(size[0], size[1], seed)
    return sc, cams, kt


def test_partial_depth_matches_oracle():
    needs_gpu()
    tile = (16, 16)
    sc, cams, kt = _merged_setup(tile, B=4, size=(61, 47))
    r = Rasterizer(tile)
    g = GaussianTensors.from_scene(sc)
    off, pix = r.subsample(cams, kt)
    _, fr = r.forward_partial(g, cams, off, pix, L.MVGS_PARTIAL_COMPACT)
    dep = r.export_depth(fr)
    torch.cuda.synchronize()
    sel = _sel_lists(off, pix, cams, tile)
    for v, c in enumerate(cams):
        xs, ys = sel[v] % c.width, sel[v] // c.width
        rgb, tf, fl, dz = oracle.render_pixels(sc, cams, v, xs, ys, with_depth=True)
        got = dep[v].cpu().numpy().astype(np.float64)[ys, xs]
        ok = fl == 0
        assert np.all(np.abs(got - dz)[ok] <= 1e-5 * np.abs(dz)[ok] + 1e-6), v
    # depth is rendered by thread-efficient frames only
    _, fm = r.forward_partial(g, cams, off, pix, L.MVGS_PARTIAL_MASKED)
    with pytest.raises(L.MvgsError):
        r.export_depth(fm)
    r.release(fm)
    r.release(fr)
    r.close()


@pytest.mark.parametrize("w", [(0.8, 0.2), (0.0, 1.0), (1.0, 0.0)])
def test_loss3d_matches_oracle(w):
    needs_gpu()
    tile = (16, 16)
    sc, cams, kt = _merged_setup(tile)
    W, H = cams[0].width, cams[0].height
    r = Rasterizer(tile)
    g = GaussianTensors.from_scene(sc)
    off, pix = r.subsample(cams, kt)
    merged = torch.zeros((3, H, W), device="cuda")
    _, fr = r.forward_partial(g, cams, off, pix, L.MVGS_PARTIAL_COMPACT, images=[merged] * len(cams))
    target = torch.rand((3, H, W), device="cuda", generator=torch.Generator(device="cuda").manual_seed(5))
    loss, grad = r.loss_3d(fr, merged, target, *w)
    # the oracle takes the same inputs: merged image, target, and points from the rendered depth and T
    plane_t = torch.ones((H, W), device="cuda")
    plane_d = torch.zeros((H, W), device="cuda")
    L.check(r.lib.mvgs_export_transmittance(r.ctx, None, fr.handle, L.ptr_array([plane_t.data_ptr()] * len(cams))),
            r.ctx)
    r.export_depth(fr, outs=[plane_d] * len(cams))
    torch.cuda.synchronize()
    sel = _sel_lists(off, pix, cams, tile)
    vm = np.zeros(W * H, int)
    for v in range(len(cams)):
        vm[sel[v]] = v
    P, S = oracle.surface_points(cams, vm.reshape(H, W), plane_d.cpu().numpy().astype(np.float64),
                                 plane_t.cpu().numpy().astype(np.float64))
    assert (S > 0).mean() > 0.5
    lo, go, _ = oracle.loss3d(merged.cpu().numpy(), target.cpu().numpy(), P, S, *w)
    assert abs(float(loss.item()) - lo) <= 1e-5 * abs(lo) + 1e-7
    gd = grad.cpu().numpy().astype(np.float64)
    assert np.allclose(gd, go, rtol=1e-4, atol=1e-5 * np.abs(go).max())
    # the gradient drives the backward like any image gradient (one plane for every view)
    grads = r.backward(g, fr, [grad] * len(cams))
    torch.cuda.synchronize()
    assert all(bool(torch.isfinite(t).all()) for t in grads.values())
    r.release(fr)
    r.close()


def test_loss3d_needs_a_plane_partition():
    needs_gpu()
    tile = (32, 32)
    sc = scenes.make_scene(3000, 1, log_scale_mean=-3.1)
    cams = scenes.make_cameras([(61, 47), (61, 47)])
    r = Rasterizer(tile, 4)
    g = GaussianTensors.from_scene(sc)
    off, pix = _uneven_selection(cams, tile, 3)
    img = torch.zeros((3, 47, 61), device="cuda")
    _, fr = r.forward_partial(g, cams, off, pix, L.MVGS_PARTIAL_COMPACT)
    with pytest.raises(L.MvgsError) as ei:
        r.loss_3d(fr, img, img)
    assert ei.value.status == L.MVGS_EINVAL
    r.release(fr)
    _, ff = r.forward(g, cams)
    with pytest.raises(L.MvgsError):
        r.loss_3d(ff, img, img)
    r.release(ff)
    r.close()
