"""The training loop's kernels on the GPU, through the C ABI: the Adam step against the oracle's,
the state gather and the gradient moments against plain numpy on seeded data, the selection merge
against the oracle's partition, the mini-batch gradient variance (Sec. 3.2) of whole-view and
partial batches against the oracle's, the finite-population law at a larger size, and a short
multi-view training run with adaptive density control that lowers the loss."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from paper_2506_12727_amd import _lib as L
from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer
from paper_2506_12727_amd.train import Trainer, variance_partial, variance_views

from gpu_common import needs_gpu

pytestmark = pytest.mark.gpu

LR = dict(means=0.01, scales=0.02, quats=0.03, opacities=0.05, sh_dc=0.004, sh_rest=0.0007)
F32 = lambda x: float(np.float32(x))
LR32 = {k: F32(v) for k, v in LR.items()}
cuda = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_adam_matches_oracle():
    needs_gpu()
    P, deg = 1000, 3
    K = (deg + 1) ** 2
    sc = scenes.make_scene(P, deg, seed=21, log_scale_mean=-3.0)
    sc.opacities[:3] = np.array([0.0, 1.0, 0.999], np.float32)
    g = GaussianTensors.from_scene(sc)
    mom = torch.zeros((P, 11 + 3 * K, 2), device="cuda")
    p = dict(means=sc.means, scales=sc.scales, quats=sc.quats, opacities=sc.opacities.reshape(-1), sh=sc.sh)
    om = np.zeros((P, 11 + 3 * K, 2))
    rng = np.random.default_rng(22)
    r = Rasterizer()
    for step in (1, 2, 3):
        gr = dict(means=rng.normal(size=(P, 3)), scales=rng.normal(size=(P, 3)), quats=rng.normal(size=(P, 4)),
                  opacities=rng.normal(size=P), sh=rng.normal(size=(P, K, 3)))
        gr = {k: v.astype(np.float32) for k, v in gr.items()}
        r.adam_step(g, {k: cuda(v) for k, v in gr.items()}, mom, step, LR)
        # the oracle takes the hyper-parameters the kernel receives (single-precision values)
        p, om = oracle.adam_step(p, gr, om, step, LR32, beta1=F32(0.9), beta2=F32(0.999), eps=F32(1e-15))
    torch.cuda.synchronize()
    for name, t in (("means", g.means), ("scales", g.scales), ("quats", g.quats), ("opacities", g.opacities),
                    ("sh", g.sh)):
        got = t.cpu().numpy().astype(np.float64)
        assert np.allclose(got, p[name], rtol=2e-6, atol=2e-6), name
    assert g.opacities[0].item() == 0.0 and g.opacities[1].item() == 1.0
    # m is a sum of terms of either sign (absolute error on the scale of the gradients); v is not
    mg = mom.cpu().numpy().astype(np.float64)
    assert np.allclose(mg[..., 0], om[..., 0], rtol=1e-5, atol=1e-6)
    assert np.allclose(mg[..., 1], om[..., 1], rtol=1e-5, atol=1e-12)
    r.close()


def test_adam_counted_on_the_device():
    """Adam with its step number counted on the device equals the host-counted step, and a void
    capacity-mode frame as skip word leaves parameters, moments and counter alone."""
    needs_gpu()
    P, deg = 700, 2
    K = (deg + 1) ** 2
    sc = scenes.make_scene(P, deg, seed=23, log_scale_mean=-3.0)
    ga, gb = GaussianTensors.from_scene(sc), GaussianTensors.from_scene(sc)
    ma = torch.zeros((P, 11 + 3 * K, 2), device="cuda")
    mb = torch.zeros_like(ma)
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    rng = np.random.default_rng(24)
    r = Rasterizer()
    for t in (1, 2, 3, 4):
        gr = dict(means=rng.normal(size=(P, 3)), scales=rng.normal(size=(P, 3)), quats=rng.normal(size=(P, 4)),
                  opacities=rng.normal(size=P), sh=rng.normal(size=(P, K, 3)))
        gr = {k: cuda(v.astype(np.float32)) for k, v in gr.items()}
        r.adam_step(ga, gr, ma, t, LR)
        r.adam_step(gb, gr, mb, 0, LR, step_dev=step)
    torch.cuda.synchronize()
    assert int(step.item()) == 4
    for name in ("means", "scales", "quats", "opacities", "sh"):
        a, b = getattr(ga, name), getattr(gb, name)
        assert torch.allclose(a, b, rtol=1e-6, atol=1e-7), name
    assert torch.allclose(ma, mb, rtol=1e-6, atol=1e-9)
    # a void frame: records over a tiny capacity
    cams = scenes.make_cameras([(64, 48)], seed=3)
    small = Rasterizer(capacity=(1, 1))
    _, fr = small.forward(ga, cams)
    with pytest.raises(L.MvgsError):
        fr.check()
    before = {n: getattr(gb, n).clone() for n in ("means", "scales", "quats", "opacities", "sh")}
    mb0 = mb.clone()
    r.adam_step(gb, gr, mb, 0, LR, step_dev=step, skip=fr)
    torch.cuda.synchronize()
    assert int(step.item()) == 4 and torch.equal(mb, mb0)
    for n, v in before.items():
        assert torch.equal(getattr(gb, n), v), n
    small.release(fr)
    small.close()
    r.close()


def test_gather_rows_and_moments():
    needs_gpu()
    rng = np.random.default_rng(23)
    x = rng.normal(size=(513, 7, 2)).astype(np.float32)
    src = rng.integers(0, 513, size=1100).astype(np.int32)
    r = Rasterizer()
    out = r.gather_rows(cuda(src), cuda(x))
    assert np.array_equal(out.cpu().numpy(), x[src])
    assert r.gather_rows(cuda(src[:0]), cuda(x)).shape == (0, 7, 2)
    # moments of five seeded "gradients"
    P, deg = 300, 1
    K = 4
    g = GaussianTensors.from_scene(scenes.make_scene(P, deg))
    s = torch.zeros(P * (11 + 3 * K), dtype=torch.float64, device="cuda")
    acc = torch.zeros(2, dtype=torch.float64, device="cuda")
    vecs = []
    for _ in range(5):
        gr = dict(means=rng.normal(size=(P, 3)), scales=rng.normal(size=(P, 3)), quats=rng.normal(size=(P, 4)),
                  opacities=rng.normal(size=P), sh=rng.normal(size=(P, K, 3)))
        gr = {k: v.astype(np.float32) for k, v in gr.items()}
        vecs.append(oracle.flatten_grads(gr))
        r.grad_moments(g, {k: cuda(v) for k, v in gr.items()}, s, acc)
    torch.cuda.synchronize()
    v = np.array(vecs)
    assert np.allclose(s.cpu().numpy(), v.sum(0), rtol=1e-12, atol=1e-12)
    a = acc.cpu().numpy()
    assert abs(a[0] - (v * v).sum()) < 1e-10 * (v * v).sum()
    assert abs(a[1] - (v.sum(0) ** 2).sum()) < 1e-10 * (v.sum(0) ** 2).sum()
    r.close()


@pytest.mark.parametrize("mode", [L.MVGS_PARTIAL_COMPACT, L.MVGS_PARTIAL_MASKED])
def test_merge_follows_the_partition(mode):
    needs_gpu()
    W, H, B, tile = 53, 37, 3, (16, 16)
    cams = scenes.make_cameras([(W, H)] * B)
    keys = np.random.default_rng(24).integers(0, 2 ** 32, size=W * H, dtype=np.uint64).astype(np.uint32)
    planes = [np.random.default_rng(30 + v).normal(size=(2, H, W)).astype(np.float32) for v in range(B)]
    r = Rasterizer(tile)
    g = GaussianTensors.from_scene(scenes.make_scene(200, 0))
    off, pix = r.subsample(cams, cuda(keys.view(np.int32)))
    _, fr = r.forward_partial(g, cams, off, pix, mode)
    out = r.merge(fr, [cuda(p) for p in planes], out=torch.full((2, H, W), -5.0, device="cuda"))
    torch.cuda.synchronize()
    o_off, o_pix = oracle.subsample_tiles(W, H, B, tile, keys)
    T = (len(o_off) - 1) // B
    want = np.full((2, H * W), -5.0, np.float32)
    for v in range(B):
        sel = o_pix[o_off[v * T]:o_off[(v + 1) * T]]
        want[:, sel] = planes[v].reshape(2, -1)[:, sel]
    assert np.array_equal(out.cpu().numpy().reshape(2, -1), want)
    r.release(fr)
    _, ff = r.forward(g, cams)
    with pytest.raises(L.MvgsError):
        r.merge(ff, [cuda(p) for p in planes])
    r.release(ff)
    r.close()


def _tiny(N=5, W=24, H=20):
    sc = scenes.make_scene(60, 1, log_scale_mean=-2.2)
    cams = scenes.make_cameras([(W, H)] * N, seed=11)
    targets = scenes.make_targets(cams, seed=12)
    return sc, cams, targets


def test_variance_of_view_batches_matches_oracle():
    needs_gpu()
    sc, cams, targets = _tiny()
    batches = [[v] for v in range(5)] + [list(s) for s in itertools.combinations(range(5), 2)]
    r = Rasterizer()
    g = GaussianTensors.from_scene(sc)
    tt = [cuda(t) for t in targets]
    for group in (batches[:5], batches[5:]):
        got = variance_views(r, g, cams, tt, group)
        want = oracle.minibatch_variance([oracle.flatten_grads(oracle.batch_gradient(sc, cams, targets, b))
                                          for b in group])
        assert abs(got["variance"] - want) <= 2e-3 * want, (got, want)
    r.close()


def test_variance_of_partial_batches_matches_oracle():
    needs_gpu()
    sc, cams, targets = _tiny()
    rng = np.random.default_rng(25)
    batches = [list(rng.choice(5, size=3, replace=False)) for _ in range(6)]
    keys = [rng.integers(0, 2 ** 32, size=24 * 20, dtype=np.uint64).astype(np.uint32) for _ in batches]
    r = Rasterizer()
    g = GaussianTensors.from_scene(sc)
    got = variance_partial(r, g, cams, [cuda(t) for t in targets], batches, [cuda(k.view(np.int32)) for k in keys])
    want = oracle.minibatch_variance([oracle.flatten_grads(oracle.partial_batch_gradient(sc, cams, targets, b, k))
                                      for b, k in zip(batches, keys)])
    assert abs(got["variance"] - want) <= 2e-3 * want, (got, want)
    r.close()


def test_sampling_law_at_a_larger_size():
    """Over all 4-subsets of 8 views the variance of the batch mean is the single-view variance
    times (N - B) / (B (N - 1)) = 1/7."""
    needs_gpu()
    sc = scenes.make_scene(20000, 3, log_scale_mean=-3.5)
    cams = scenes.make_cameras([(160, 120)] * 8, seed=14)
    tt = [cuda(t) for t in scenes.make_targets(cams, seed=15)]
    r = Rasterizer()
    g = GaussianTensors.from_scene(sc)
    v1 = variance_views(r, g, cams, tt, [[v] for v in range(8)])["variance"]
    v4 = variance_views(r, g, cams, tt, [list(s) for s in itertools.combinations(range(8), 4)])["variance"]
    assert abs(v4 - v1 / 7) <= 1e-3 * v1 / 7, (v1, v4)
    r.close()


def _problem(P=3000, N=12, size=(64, 64), seed=31):
    gt_sc = scenes.make_scene(P, 1, seed=seed, log_scale_mean=-3.2)
    init = scenes.make_scene(P, 1, seed=seed, log_scale_mean=-3.2)
    rng = np.random.default_rng(seed + 1)
    init.means += rng.normal(0.0, 0.03, size=init.means.shape).astype(np.float32)
    init.sh[:] = rng.normal(0.0, 0.2, size=init.sh.shape).astype(np.float32)
    cams = scenes.make_cameras([size] * N, seed=seed + 2)
    return GaussianTensors.from_scene(init), GaussianTensors.from_scene(gt_sc), cams


@pytest.mark.parametrize("partial", [False, True])
def test_training_lowers_the_loss_and_densifies(partial):
    needs_gpu()
    g, gt, cams = _problem()
    lr = dict(means=1e-3, scales=5e-3, quats=1e-3, opacities=2e-2, sh_dc=1e-2, sh_rest=2e-3)
    t = Trainer(g, gt, cams, views_per_step=4, partial=partial, lr=lr, w_l1=0.8, w_dssim=0.2,
                densify=dict(split_threshold=1e-7, clone_threshold=1e-7), densify_from=30, densify_until=61,
                densify_every=30, seed=5)
    P0 = t.g.P
    losses = t.run(150)
    assert all(np.isfinite(losses))
    assert t.n_densified == 2 and t.g.P != P0
    for name in ("means", "scales", "quats", "opacities", "sh"):
        assert bool(torch.isfinite(getattr(t.g, name)).all()), name
    assert np.mean(losses[-10:]) < 0.8 * np.mean(losses[:10]), (losses[:10], losses[-10:])
    t.close()


@pytest.mark.parametrize("partial", [False, True])
def test_captured_training_matches_eager(partial):
    """The training loop as one graph replay per iteration (Adam counted on the device, density
    control between captures) follows the eager loop: the same first loss, losses that stay close
    (float atomics make the runs drift apart slowly) and the same density control decisions on
    the first round; it lowers the loss like the eager loop."""
    needs_gpu()
    lr = dict(means=1e-3, scales=5e-3, quats=1e-3, opacities=2e-2, sh_dc=1e-2, sh_rest=2e-3)
    runs = {}
    for captured in (False, True):
        g, gt, cams = _problem()
        t = Trainer(g, gt, cams, views_per_step=4, partial=partial, lr=lr, w_l1=0.8, w_dssim=0.2,
                    densify=dict(split_threshold=1e-7, clone_threshold=1e-7), densify_from=20, densify_until=41,
                    densify_every=20, seed=5, captured=captured)
        P0 = t.g.P
        losses = t.run(60)
        runs[captured] = (losses, t.g.P, t.n_densified, P0)
        for name in ("means", "scales", "quats", "opacities", "sh"):
            assert bool(torch.isfinite(getattr(t.g, name)).all()), name
        if captured:
            assert t.cstep is not None and t.recaptures == 0
        t.close()
    le, P_e, nd_e, _ = runs[False]
    lc, P_c, nd_c, _ = runs[True]
    assert nd_c == nd_e == 2
    assert all(np.isfinite(lc))
    assert np.mean(lc[-10:]) < 0.85 * np.mean(lc[:10]), (lc[:10], lc[-10:])
    if not partial:
        # the same batches from the same parameters: the first loss agrees to rounding
        assert abs(lc[0] - le[0]) <= 1e-6 * abs(le[0])
        assert np.allclose(lc[:20], le[:20], rtol=2e-2), (lc[:20], le[:20])
        assert abs(P_c - P_e) <= 0.02 * P_e
    else:
        # keys come from different generators: compare the trajectories on average
        assert abs(np.mean(lc[-10:]) - np.mean(le[-10:])) <= 0.1 * np.mean(le[-10:])
