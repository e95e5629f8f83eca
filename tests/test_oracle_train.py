"""The oracle's pieces of the training loop, pinned: the Adam step against torch.optim.Adam (a
library implementation) and the closed form of a constant gradient; the Monte Carlo variance of
Sec. 3.2 against numpy's variance; the mini-batch gradients against the finite-population law of
sampling views without replacement and against a full render for partial batches of one camera."""
import itertools

import numpy as np
import torch

import oracle
from paper_2506_12727_amd import scenes

LR = dict(means=0.01, scales=0.02, quats=0.03, opacities=0.05, sh_dc=0.004, sh_rest=0.0007)


def _params(P, K, seed):
    rng = np.random.default_rng(seed)
    return dict(means=rng.normal(size=(P, 3)), scales=rng.uniform(0.01, 0.2, size=(P, 3)),
                quats=rng.normal(size=(P, 4)), opacities=rng.uniform(0.02, 0.98, size=P),
                sh=rng.normal(size=(P, K, 3)))


def _grads(P, K, rng):
    return dict(means=rng.normal(size=(P, 3)), scales=rng.normal(size=(P, 3)), quats=rng.normal(size=(P, 4)),
                opacities=rng.normal(size=P), sh=rng.normal(size=(P, K, 3)))


def test_adam_matches_torch_adam():
    P, K = 7, 4
    p0 = _params(P, K, 1)
    rng = np.random.default_rng(2)
    seq = [_grads(P, K, rng) for _ in range(4)]
    # torch's Adam on the unconstrained coordinates, one group per learning rate
    t = dict(means=torch.tensor(p0["means"], requires_grad=True),
             log_s=torch.tensor(np.log(p0["scales"]), requires_grad=True),
             quats=torch.tensor(p0["quats"], requires_grad=True),
             logit=torch.tensor(np.log(p0["opacities"] / (1 - p0["opacities"])), requires_grad=True),
             dc=torch.tensor(p0["sh"][:, :1].copy(), requires_grad=True),
             rest=torch.tensor(p0["sh"][:, 1:].copy(), requires_grad=True))
    opt = torch.optim.Adam([dict(params=[t["means"]], lr=LR["means"]), dict(params=[t["log_s"]], lr=LR["scales"]),
                            dict(params=[t["quats"]], lr=LR["quats"]), dict(params=[t["logit"]], lr=LR["opacities"]),
                            dict(params=[t["dc"]], lr=LR["sh_dc"]), dict(params=[t["rest"]], lr=LR["sh_rest"])],
                           betas=(0.9, 0.999), eps=1e-15)
    p, mom = p0, np.zeros((P, 11 + 3 * K, 2))
    for step, gr in enumerate(seq, start=1):
        with torch.no_grad():
            s = torch.exp(t["log_s"])
            o = torch.sigmoid(t["logit"])
        # gradients with respect to the activated values, passed through the activations
        t["means"].grad = torch.tensor(gr["means"])
        t["log_s"].grad = torch.tensor(gr["scales"]) * s
        t["quats"].grad = torch.tensor(gr["quats"])
        t["logit"].grad = torch.tensor(gr["opacities"]) * o * (1 - o)
        t["dc"].grad = torch.tensor(gr["sh"][:, :1].copy())
        t["rest"].grad = torch.tensor(gr["sh"][:, 1:].copy())
        opt.step()
        p, mom = oracle.adam_step(p, gr, mom, step, LR)
        assert np.allclose(p["means"], t["means"].detach().numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(p["scales"], np.exp(t["log_s"].detach().numpy()), rtol=1e-12)
        assert np.allclose(p["quats"], t["quats"].detach().numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(p["opacities"], torch.sigmoid(t["logit"]).detach().numpy(), rtol=1e-11)
        sh = np.concatenate([t["dc"].detach().numpy(), t["rest"].detach().numpy()], axis=1)
        assert np.allclose(p["sh"], sh, rtol=1e-12, atol=1e-14)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are the gradient and its square at
    every step, so each step moves by lr * sign(g) (eps aside)."""
    P, K = 5, 1
    p0 = _params(P, K, 3)
    rng = np.random.default_rng(4)
    g = _grads(P, K, rng)
    p, mom = p0, np.zeros((P, 11 + 3 * K, 2))
    for step in range(1, 6):
        p, mom = oracle.adam_step(p, g, mom, step, LR)
    assert np.allclose(p["means"], p0["means"] - 5 * LR["means"] * np.sign(g["means"]), rtol=1e-12, atol=1e-13)
    assert np.allclose(p["quats"], p0["quats"] - 5 * LR["quats"] * np.sign(g["quats"]), rtol=1e-12, atol=1e-13)
    assert np.allclose(p["sh"][:, 0], p0["sh"][:, 0] - 5 * LR["sh_dc"] * np.sign(g["sh"][:, 0]), atol=1e-13)
    # first step of a scale and an opacity: their log / logit move by lr against the gradient's sign
    p1, _ = oracle.adam_step(p0, g, np.zeros((P, 11 + 3 * K, 2)), 1, LR)
    assert np.allclose(np.log(p1["scales"] / p0["scales"]), -LR["scales"] * np.sign(g["scales"]), rtol=1e-10)
    lg = lambda o: np.log(o / (1 - o))
    assert np.allclose(lg(p1["opacities"]) - lg(p0["opacities"]), -LR["opacities"] * np.sign(g["opacities"]),
                       rtol=1e-9)


def test_adam_keeps_saturated_opacities():
    P, K = 3, 1
    p0 = _params(P, K, 5)
    p0["opacities"] = np.array([0.0, 1.0, 0.5])
    g = _grads(P, K, np.random.default_rng(6))
    p1, _ = oracle.adam_step(p0, g, np.zeros((P, 11 + 3 * K, 2)), 1, LR)
    assert p1["opacities"][0] == 0.0 and p1["opacities"][1] == 1.0 and 0 < p1["opacities"][2] < 1


def test_minibatch_variance_is_numpys_variance():
    x = np.random.default_rng(7).normal(size=(40, 13)) * np.arange(1, 14)
    assert abs(oracle.minibatch_variance(x) - float(np.var(x, axis=0).sum())) < 1e-10 * float(np.var(x, axis=0).sum())


def _tiny(N=5, W=24, H=20):
    sc = scenes.make_scene(60, 1, log_scale_mean=-2.2)
    cams = scenes.make_cameras([(W, H)] * N, seed=11)
    targets = scenes.make_targets(cams, seed=12)
    return sc, cams, targets


def test_view_batches_follow_the_sampling_law():
    """Over every B-subset of N views, the variance of the mean of B view gradients is the
    single-view variance times (N - B) / (B (N - 1)): the batch gradient must be the mean of the
    views' gradients and the estimator the variance of Sec. 3.2."""
    sc, cams, targets = _tiny()
    N = len(cams)
    single = [oracle.flatten_grads(oracle.batch_gradient(sc, cams, targets, [v])) for v in range(N)]
    v1 = oracle.minibatch_variance(single)
    assert v1 > 0
    for B in (2, 3):
        subsets = list(itertools.combinations(range(N), B))
        vb = oracle.minibatch_variance([oracle.flatten_grads(oracle.batch_gradient(sc, cams, targets, list(s)))
                                        for s in subsets])
        assert abs(vb - v1 * (N - B) / (B * (N - 1))) < 1e-9 * v1
    # the full batch has no variance
    assert abs(oracle.minibatch_variance([oracle.flatten_grads(oracle.batch_gradient(sc, cams, targets,
                                                                                     list(range(N))))])) < 1e-20


def test_partial_batch_of_one_camera_is_the_full_view():
    """B copies of one camera sharing its image plane cover every pixel once: the partial batch
    gradient is that view's whole-image gradient."""
    sc, cams, targets = _tiny(N=1)
    keys = np.random.default_rng(13).integers(0, 2 ** 32, size=24 * 20, dtype=np.uint64).astype(np.uint32)
    same = [cams[0]] * 3
    tg = [targets[0]] * 3
    a = oracle.flatten_grads(oracle.partial_batch_gradient(sc, same, tg, [0, 1, 2], keys))
    b = oracle.flatten_grads(oracle.batch_gradient(sc, cams, targets, [0]))
    assert np.allclose(a, b, rtol=1e-10, atol=1e-14 * np.abs(b).max())
