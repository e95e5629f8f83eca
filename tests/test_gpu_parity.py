"""Parity of the HIP path with the CPU oracle, through the C ABI.

Binning (keys, values, ranges, counts) bit for bit; images and final transmittance within
1e-5 relative + 1e-6 absolute outside pixels the oracle flags (a cut, clamp or transmittance-stop
decision, taken in double precision by the oracle, that lies within the kernel's single-precision
error of its threshold; under 0.1% of pixels); loss and image gradients; parameter gradients and
densification statistics against the oracle's double-precision geometry within 1e-3 relative
(elementwise, plus 1e-4 of the largest magnitude; and 1e-3 in relative L2), with flagged pixels'
image gradients zero on both sides.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer

from gpu_common import (FLAG_MAX, compare_grad, compare_images, flag_fraction, grad_flags, needs_gpu, run_forward,
                        to_np, zero_flagged)

pytestmark = pytest.mark.gpu


def _small():
    return scenes.WORKLOADS["small_16k_4x128"]


def _ragged(deg=3, lsm=-3.0):
    return (scenes.make_scene(6000, deg, log_scale_mean=lsm), scenes.make_cameras([(61, 47), (130, 70), (33, 97)]))


# name -> (scene, cameras, tile, pixels per lane)
CASES = {
    # the small benchmark workload: 16,384 Gaussians, SH 0, 4 x 128^2, 16x16 tiles
    "small": lambda: (_small().scene(), _small().cameras(), (16, 16), 0),
    # ragged views and SH 3 with larger splats, several tile shapes and lane layouts
    "ragged_16x16": lambda: _ragged() + ((16, 16), 2),
    "ragged_16x16_ppl1": lambda: _ragged() + ((16, 16), 1),
    "ragged_8x8": lambda: _ragged() + ((8, 8), 1),
    "ragged_32x16": lambda: _ragged(2, -3.2) + ((32, 16), 2),
    "ragged_16x32_ppl4": lambda: _ragged(1, -3.1) + ((16, 32), 4),
    "ragged_32x32_ppl4": lambda: _ragged(3, -2.8) + ((32, 32), 4),
    "ragged_8x32_ppl2": lambda: _ragged(3, -3.0) + ((8, 32), 2),
    # more views than the emission's LDS table of view tile bases holds (its global-memory search),
    # with records that cover few tiles each (the 1,024-record emission chunks)
    "many_views": lambda: (scenes.make_scene(3000, 1, log_scale_mean=-3.6),
                           scenes.make_cameras([(24, 20), (17, 31)] * 70, seed=23), (16, 16), 0),
    # about 9 records per Gaussian: the records of 64 Gaussians just exceed the 512-record LDS stage
    # of the records kernel (46 of 47 runs go through it in two windows)
    "nine_views": lambda: (scenes.make_scene(3000, 1, log_scale_mean=-3.0),
                           scenes.make_cameras([(64, 48)] * 9, seed=31), (16, 16), 0),
    # 12 records per Gaussian: every run of 64 Gaussians (762-768 records) is written directly
    "twelve_views": lambda: (scenes.make_scene(3008, 1, log_scale_mean=-2.6),
                             scenes.make_cameras([(64, 48)] * 12, seed=5), (16, 16), 0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_binning_bit_exact(case):
    needs_gpu()
    sc, cams, tile, ppl = CASES[case]()
    r, g, imgs, fr = run_forward(sc, cams, tile, ppl=ppl)
    keys, vals, ranges = r.export_binning(fr)
    ok, ov, orr = oracle.binning(sc, cams, tile)
    gk = keys.cpu().numpy().view(np.uint64)
    assert len(gk) == len(ok) > 0
    assert np.array_equal(gk, ok)
    assert np.array_equal(vals.cpu().numpy().view(np.uint32), ov)
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), orr)
    recs, pairs = oracle.count_pairs(sc, cams, tile)
    info = fr.info()
    assert (info["records"], info["pairs"]) == (recs, pairs)
    r.release(fr)


def _depth_case(kind):
    """A camera looking along +z from z = -3 (depth = z + 3) over Gaussians all at z = 0 (every
    depth key equal: the depth sort orders one bit, ties only), or spread from depth 0.3 to 500
    (keys that differ in 27 bits: four passes)."""
    sc = scenes.make_scene(3000, 1, seed=17, log_scale_mean=-3.0)
    rng = np.random.default_rng(18)
    if kind == "equal":
        sc.means[:, 2] = 0.0
    else:
        sc.means[:, 2] = (np.exp(rng.uniform(np.log(0.3), np.log(500.0), size=len(sc.means))) - 3.0)
        sc.means[:, :2] *= (sc.means[:, 2:3] + 3.0) / 3.0   # keep them in view
    sc.means = sc.means.astype(np.float32)
    f = 0.5 * 96 / np.tan(np.radians(30.0))
    cams = [scenes.Camera(96, 80, float(np.float32(f)), float(np.float32(f)), 48.0, 40.0,
                          np.eye(3, dtype=np.float32), np.array([0.0, 0.0, 3.0], np.float32))]
    return sc, cams


@pytest.mark.parametrize("kind", ["equal", "wide"])
def test_depth_sort_key_range_edges(kind):
    """The depth sort orders only the bits in which the records' depth keys differ (eager), or a
    window of them (capacity mode, after a check): binning stays bit for bit the oracle's at both
    ends of the range."""
    needs_gpu()
    sc, cams = _depth_case(kind)
    ok, ov, orr = oracle.binning(sc, cams, (16, 16))
    assert len(ok) > 100

    def same(r, fr):
        keys, vals, ranges = r.export_binning(fr)
        assert np.array_equal(keys.cpu().numpy().view(np.uint64), ok)
        assert np.array_equal(vals.cpu().numpy().view(np.uint32), ov)
        assert np.array_equal(ranges.cpu().numpy().view(np.uint32), orr)

    r, g, imgs, fr = run_forward(sc, cams, (16, 16))
    same(r, fr)
    r.release(fr)
    info_r = oracle.count_pairs(sc, cams, (16, 16))
    cap = Rasterizer((16, 16), capacity=(info_r[0] + 10, info_r[1] + 10))
    for _ in range(2):   # the second call sorts the window the first call's check set
        _, fc = cap.forward(g, cams)
        fc.check()
        same(cap, fc)
        cap.release(fc)
    cap.close()
    r.close()


@pytest.mark.parametrize("case", list(CASES))
def test_forward_images(case):
    needs_gpu()
    sc, cams, tile, ppl = CASES[case]()
    r, g, imgs, fr = run_forward(sc, cams, tile, ppl=ppl)
    ref = oracle.forward(sc, cams, tile)
    frac = compare_images(to_np(imgs), ref["images"], ref["flags"])
    tf = to_np(r.export_transmittance(fr))
    compare_images(tf, ref["t_final"], ref["flags"])
    print(f"{case}: flagged pixels {frac:.2e}")
    assert frac < FLAG_MAX
    r.release(fr)


@pytest.mark.parametrize("w", [(1.0, 0.0), (0.8, 0.2), (0.0, 1.0)])
def test_loss_and_image_gradient(w):
    needs_gpu()
    # ragged views spanning several 32x32 loss tiles, views smaller than one tile, 1x1 and 1-wide
    cams = scenes.make_cameras([(61, 47), (40, 90), (16, 16), (97, 70), (1, 1), (1, 37), (5, 3), (64, 32)])
    rng = np.random.default_rng(7)
    imgs = [rng.uniform(size=(3, c.height, c.width)).astype(np.float32) for c in cams]
    tg = scenes.make_targets(cams)
    r = Rasterizer()
    gi = [torch.from_numpy(a).cuda() for a in imgs]
    gt = [torch.from_numpy(a).cuda() for a in tg]
    loss, grads = r.loss(cams, gi, gt, *w)
    lo, go = oracle.loss(cams, imgs, tg, *w)
    assert abs(float(loss.item()) - lo) <= 1e-5 * abs(lo) + 1e-7
    for a, b in zip(to_np(grads), go):
        assert np.allclose(a, b, rtol=1e-4, atol=1e-5 * np.abs(b).max())


def _backward_case(sc, cams, tile, w_l1, w_dssim, densify, ppl=0):
    r, g, imgs, fr = run_forward(sc, cams, tile, ppl=ppl)
    flags = grad_flags(sc, cams, tile)
    frac = flag_fraction(flags)
    print(f"gradient parity: flagged pixels {frac:.2e}")
    assert frac < FLAG_MAX
    tg = [torch.from_numpy(a).cuda() for a in scenes.make_targets(cams)]
    _, dl = r.loss(cams, imgs, tg, w_l1, w_dssim)
    # pixels where a decision of the double-precision walk may go the other way in the kernel
    # contribute to neither side
    zero_flagged(dl, flags)
    P = g.P
    dz = None
    if densify:
        dz = dict(e1=torch.zeros(P, device="cuda"), e2=torch.zeros(P, device="cuda"),
                  count=torch.zeros(P, dtype=torch.int32, device="cuda"))
    grads = r.backward(g, fr, dl, densify=dz)
    torch.cuda.synchronize()
    ob = oracle.backward(sc, cams, to_np(dl), tile, geom32_mode=False)
    out = {}
    for n in ("means", "scales", "quats", "opacities", "sh"):
        out[n] = compare_grad(n, grads[n].cpu().numpy(), ob[n])
    if densify:
        out["e1"] = compare_grad("e1", dz["e1"].cpu().numpy(), ob["e1"])
        out["e2"] = compare_grad("e2", dz["e2"].cpu().numpy(), ob["e2"])
        assert np.array_equal(dz["count"].cpu().numpy(), ob["count"])
    r.release(fr)
    return out


@pytest.mark.parametrize("case", list(CASES))
def test_backward_gradients_and_statistics(case):
    needs_gpu()
    sc, cams, tile, ppl = CASES[case]()
    _backward_case(sc, cams, tile, 1.0, 0.0, densify=True, ppl=ppl)


def test_backward_with_dssim():
    needs_gpu()
    sc = scenes.make_scene(5000, 3, log_scale_mean=-3.2)
    cams = scenes.make_cameras([(96, 64), (64, 96)])
    _backward_case(sc, cams, (16, 16), 0.8, 0.2, densify=False)


def test_statistics_accumulate_across_calls():
    needs_gpu()
    sc, cams, tile, ppl = CASES["small"]()
    r, g, imgs, fr = run_forward(sc, cams, tile, ppl=ppl)
    tg = [torch.from_numpy(a).cuda() for a in scenes.make_targets(cams)]
    _, dl = r.loss(cams, imgs, tg, 1.0, 0.0)
    P = g.P
    dz = dict(e1=torch.zeros(P, device="cuda"), e2=torch.zeros(P, device="cuda"),
              count=torch.zeros(P, dtype=torch.int32, device="cuda"))
    r.backward(g, fr, dl, densify=dz)
    once = {k: v.clone() for k, v in dz.items()}
    r.backward(g, fr, dl, densify=dz)
    torch.cuda.synchronize()
    assert torch.equal(dz["count"], 2 * once["count"])
    assert torch.allclose(dz["e1"], 2 * once["e1"], rtol=1e-5, atol=0)
    # E_old <= E2 <= E1 per Gaussian (triangle inequality), up to rounding
    assert bool((once["e2"] <= once["e1"] * (1 + 1e-4) + 1e-12).all())
    r.release(fr)


def test_backward_reuses_cleared_accumulators():
    """Repeated backwards on one context (the per-record accumulators reused), a larger batch
    (the buffer grows) and a smaller one afterwards all equal the same backward on a fresh
    context."""
    needs_gpu()
    sc = scenes.make_scene(8000, 3, log_scale_mean=-3.2)
    small = scenes.make_cameras([(61, 47), (130, 70)], seed=5)
    big = scenes.make_cameras([(61, 47), (130, 70), (160, 96), (96, 128)], seed=6)
    g = GaussianTensors.from_scene(sc)
    r = Rasterizer()

    def grads_of(rast, cams, seed):
        imgs, fr = rast.forward(g, cams)
        dl = [torch.from_numpy(np.random.default_rng(seed + v).standard_normal((3, c.height, c.width))
                               .astype(np.float32)).cuda() for v, c in enumerate(cams)]
        dz = dict(e1=torch.zeros(g.P, device="cuda"), e2=torch.zeros(g.P, device="cuda"),
                  count=torch.zeros(g.P, dtype=torch.int32, device="cuda"))
        out = rast.backward(g, fr, dl, densify=dz)
        torch.cuda.synchronize()
        rast.release(fr)
        return {k: v.clone() for k, v in out.items()}, dz

    for cams, seed in ((small, 1), (small, 2), (big, 3), (big, 4), (small, 5)):
        got, dz = grads_of(r, cams, seed)
        fresh = Rasterizer()
        ref, dz_ref = grads_of(fresh, cams, seed)
        fresh.close()
        for n in ref:
            compare_grad(n, got[n].cpu().numpy(), ref[n].cpu().numpy().astype(np.float64), rtol=1e-4, inf=1e-5,
                         l2=1e-4)
        assert torch.equal(dz["count"], dz_ref["count"])
        compare_grad("e1", dz["e1"].cpu().numpy(), dz_ref["e1"].cpu().numpy().astype(np.float64), rtol=1e-4,
                     inf=1e-5, l2=1e-4)
    r.close()


def test_batch_invariance_and_rerun_determinism():
    """A view rendered alone equals the same view rendered inside a batch, bit for bit, and two
    runs of the same batch give identical images and binning."""
    needs_gpu()
    sc = scenes.make_scene(8000, 3, log_scale_mean=-3.2)
    cams = scenes.make_cameras([(61, 47), (130, 70), (33, 97)])
    r = Rasterizer()
    g = GaussianTensors.from_scene(sc)
    batch, fb = r.forward(g, cams)
    batch2, fb2 = r.forward(g, cams)
    for v, c in enumerate(cams):
        alone, fa = r.forward(g, [c])
        assert torch.equal(alone[0], batch[v])
        r.release(fa)
    for a, b in zip(batch, batch2):
        assert torch.equal(a, b)
    k1, v1, r1 = r.export_binning(fb)
    k2, v2, r2 = r.export_binning(fb2)
    assert torch.equal(k1, k2) and torch.equal(v1, v2) and torch.equal(r1, r2)
    r.release(fb)
    r.release(fb2)


def test_edge_cases():
    needs_gpu()
    r = Rasterizer()
    cams = scenes.make_cameras([(37, 29), (1, 1)])
    for c in cams:
        c.bg = np.array([0.25, 0.5, 0.75], np.float32)
    bg = torch.tensor([0.25, 0.5, 0.75], device="cuda")[:, None, None]
    # empty scene: background only, no pairs
    empty = scenes.make_scene(0, 0)
    g = GaussianTensors.from_scene(empty)
    imgs, fr = r.forward(g, cams)
    assert fr.info()["pairs"] == 0
    for im in imgs:
        assert torch.equal(im, bg.expand_as(im))
    tg = [torch.rand_like(i) for i in imgs]
    _, dl = r.loss(cams, imgs, tg, 1.0, 0.0)
    grads = r.backward(g, fr, dl)
    r.release(fr)
    # every Gaussian behind the cameras
    sc = scenes.make_scene(500, 1)
    cams2 = [scenes.make_camera(37, 29, (0, 0, -3.0))]
    cams2[0].bg = np.array([0.25, 0.5, 0.75], np.float32)
    sc.means[:, 2] = -5.0
    g = GaussianTensors.from_scene(sc)
    imgs, fr = r.forward(g, cams2)
    assert fr.info()["records"] == 0
    assert torch.equal(imgs[0], bg.expand_as(imgs[0]))
    _, dl = r.loss(cams2, imgs, [torch.rand_like(imgs[0])], 1.0, 0.0)
    grads = r.backward(g, fr, dl)
    torch.cuda.synchronize()
    assert all(float(t.abs().max()) == 0.0 for t in grads.values())
    r.release(fr)


def test_maximum_tiles_per_view():
    """4096 x 4096 at 16x16 tiles is exactly the 65,536-tile limit of the 16-bit tile field."""
    needs_gpu()
    sc = scenes.make_scene(4000, 0, log_scale_mean=-3.0)
    cams = [scenes.make_camera(4096, 4096, (0.0, 0.3, -2.5))]
    r, g, imgs, fr = run_forward(sc, cams)
    assert fr.info()["tiles"] == 65536
    keys, vals, ranges = r.export_binning(fr)
    ok, ov, orr = oracle.binning(sc, cams)
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ok)
    assert np.array_equal(vals.cpu().numpy().view(np.uint32), ov)
    rng = np.random.default_rng(3)
    xs, ys = rng.integers(0, 4096, 300), rng.integers(0, 4096, 300)
    rgb, tf, fl = oracle.render_pixels(sc, cams, 0, xs, ys)
    got = imgs[0].cpu().numpy().astype(np.float64)[:, ys, xs].T
    ok_ = fl == 0
    assert np.all(np.abs(got - rgb)[ok_] <= 1e-5 * np.abs(rgb)[ok_] + 1e-6)
    r.release(fr)


def test_more_tiles_than_16_bit_ids():
    """Two 2048 x 2048 views at 8x8 tiles: 131,072 tiles in the batch, so the pair keys are 32-bit
    tile ids (17 bits, three tile-sort passes); at most 65,536 tiles they are 16-bit."""
    needs_gpu()
    sc = scenes.make_scene(3000, 0, log_scale_mean=-3.2)
    cams = [scenes.make_camera(2048, 2048, (0.0, 0.3, -2.5)), scenes.make_camera(2048, 2048, (0.4, -0.2, -2.7))]
    r, g, imgs, fr = run_forward(sc, cams, (8, 8))
    assert fr.info()["tiles"] == 131072
    keys, vals, ranges = r.export_binning(fr)
    ok, ov, orr = oracle.binning(sc, cams, (8, 8))
    assert len(ok) > 0
    assert np.array_equal(keys.cpu().numpy().view(np.uint64), ok)
    assert np.array_equal(vals.cpu().numpy().view(np.uint32), ov)
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32), orr)
    rng = np.random.default_rng(5)
    for v in range(2):
        xs, ys = rng.integers(0, 2048, 300), rng.integers(0, 2048, 300)
        rgb, tf, fl = oracle.render_pixels(sc, cams, v, xs, ys)
        got = imgs[v].cpu().numpy().astype(np.float64)[:, ys, xs].T
        ok_ = fl == 0
        assert np.all(np.abs(got - rgb)[ok_] <= 1e-5 * np.abs(rgb)[ok_] + 1e-6)
    r.release(fr)
