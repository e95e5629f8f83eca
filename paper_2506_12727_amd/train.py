"""Multi-view training on synthetic scenes, and the variance of mini-batch gradients.

`Trainer` is a training loop around the rasterizer: each iteration draws a mini-batch of B views
(without replacement within an epoch), renders them (all pixels, or the thread-efficient partial
rendering of Alg. 3 where the B views share each image plane), takes the fused L1 + D-SSIM loss
(the 3D distance-aware D-SSIM of Sec. 5.1.2 for partial batches), runs the backward with the
densification statistics of Eqs. 13-14 and one Adam step. Between `densify_from` and
`densify_until`, every `densify_every` iterations it applies the multi-view adaptive density
control of Sec. 5.2.2 (split by E1, clone by E2, the pruning threshold times B as the paper's
appendix prescribes for multi-view batches), carries the optimiser moments of every Gaussian to
its outputs and clears the statistics. Targets are renders of a ground-truth scene, so the
problem has a known optimum. Every step of it runs in the library's kernels; torch holds memory
and draws the random numbers (view order, sub-sampling keys, split normals).

With `captured=True` (views of one size) an iteration is one replay of a HIP graph holding the
whole step, Adam included (step number counted on the device): the host only writes the batch's
poses, gathers its targets and replays. The capacities hold any batch of the pool with
`headroom`; the host waits for each replay (the pose staging the graph reads is host memory) and
checks it, and a step that overflowed, which changed nothing, is captured again with larger
capacities and rerun. Density control runs eagerly and the next iteration captures anew. Sub-
sampling keys are then drawn inside the graph from torch's default generator.

`variance_views` and `variance_partial` estimate the variance of mini-batch gradients over given
mini-batches (Sec. 3.2): the mean squared norm of the mini-batch gradients minus the squared
norm of their mean, accumulated on the GPU in double precision.
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .graph import CapturedStep, measure_capacity_pool
from .raster import GaussianTensors, Rasterizer

# the 3DGS learning rates (the position rate for a scene extent of about 2)
DEFAULT_LR = dict(means=3.2e-4, scales=5e-3, quats=1e-3, opacities=5e-2, sh_dc=2.5e-3, sh_rest=2.5e-3 / 20)
DEFAULT_ADC = dict(split_threshold=2e-4, clone_threshold=2e-4, dense_scale=0.02, min_opacity=0.005)


def _zeros_like_grads(g: GaussianTensors) -> dict:
    return dict(means=torch.zeros_like(g.means), scales=torch.zeros_like(g.scales), quats=torch.zeros_like(g.quats),
                opacities=torch.zeros_like(g.opacities), sh=torch.zeros_like(g.sh))


def _stats(P: int, dev) -> dict:
    return dict(e1=torch.zeros(P, device=dev), e2=torch.zeros(P, device=dev),
                count=torch.zeros(P, dtype=torch.int32, device=dev))


def _moments(g: GaussianTensors) -> torch.Tensor:
    K = (g.sh_degree + 1) ** 2
    return torch.zeros((g.P, 11 + 3 * K, 2), device=g.means.device)


class Trainer:
    def __init__(self, g: GaussianTensors, gt: GaussianTensors, cams: Sequence, views_per_step: int = 4,
                 partial: bool = False, w_l1: float = 0.8, w_dssim: float = 0.2, lr: Optional[dict] = None,
                 densify: Optional[dict] = None, densify_from: int = 100, densify_until: int = 1000,
                 densify_every: int = 100, tile=(16, 16), ppl: int = 0, seed: int = 0, captured: bool = False,
                 headroom: float = 1.3):
        g.check()
        gt.check()
        self.g = g
        self.cams = list(cams)
        self.B = int(views_per_step)
        if not 1 <= self.B <= len(self.cams):
            raise ValueError(f"views_per_step={self.B} outside [1, {len(self.cams)}]")
        self.partial = bool(partial)
        if self.partial and len({(c.width, c.height) for c in self.cams}) != 1:
            raise ValueError("partial rendering shares one image plane: the views must have one size")
        self.w_l1, self.w_dssim = float(w_l1), float(w_dssim)
        self.lr = dict(DEFAULT_LR, **(lr or {}))
        self.adc = dict(DEFAULT_ADC, **(densify or {}))
        self.densify_from, self.densify_until, self.densify_every = densify_from, densify_until, densify_every
        self.rast = Rasterizer(tile, ppl)
        self.dev = g.means.device
        self.gen = torch.Generator(device=self.dev)
        self.gen.manual_seed(seed)
        self.rng = np.random.default_rng(seed)
        self.order: List[int] = []
        # the targets: every view rendered once from the ground truth
        imgs, fr = self.rast.forward(gt, self.cams)
        self.rast.release(fr)
        self.targets = imgs
        self.moments = _moments(g)
        self.stats = _stats(g.P, self.dev)
        self.grads = _zeros_like_grads(g)
        self.it = 0
        self.n_densified = 0
        self.tile, self.ppl = tile, ppl
        self.captured, self.headroom = bool(captured), float(headroom)
        self.cstep: Optional[CapturedStep] = None
        self.recaptures = 0
        if self.captured:
            if len({(c.width, c.height) for c in self.cams}) != 1:
                raise ValueError("a captured step keeps its image sizes: the views must have one size")
            self.target_stack = torch.stack(self.targets)
            self.step_dev = torch.zeros(1, dtype=torch.int32, device=self.dev)

    def _next_views(self) -> List[int]:
        if len(self.order) < self.B:
            self.order = list(self.rng.permutation(len(self.cams)))
        views, self.order = self.order[:self.B], self.order[self.B:]
        return [int(v) for v in views]

    def _capture(self, cams, idx, capacity=None):
        """Captures the step for the current Gaussians; its warm-up call is this iteration."""
        if capacity is None:
            capacity = measure_capacity_pool(self.g, self.cams, self.B, self.tile, self.ppl, self.headroom)
        self.batch_targets = torch.index_select(self.target_stack, 0, idx)
        self.step_dev.fill_(self.it)
        self.cstep = CapturedStep(self.g, cams, list(self.batch_targets.unbind(0)), self.w_l1, self.w_dssim,
                                  tile=self.tile, ppl=self.ppl, capacity=capacity, densify=self.stats,
                                  partial=self.partial,
                                  optimizer=dict(moments=self.moments, lr=self.lr, step=self.step_dev))

    def _captured_step(self, views) -> torch.Tensor:
        cams = [self.cams[v] for v in views]
        idx = torch.as_tensor(views, dtype=torch.int64, device=self.dev)
        if self.cstep is None:
            self._capture(cams, idx)
            return self.cstep.loss
        self.cstep.set_cameras(cams)
        torch.index_select(self.target_stack, 0, idx, out=self.batch_targets)
        self.cstep.replay()
        try:
            self.cstep.check()
        except L.MvgsError as e:
            if e.status not in (L.MVGS_ECAPACITY, L.MVGS_ERETRY):
                raise
            # the replay changed nothing: capture again and rerun, with room for this batch after an
            # overflow, with the same capacities after a depth-window miss (the check moved the
            # window to this batch's keys)
            cap = self.cstep.rast.capacity
            if e.status == L.MVGS_ECAPACITY:
                cap = tuple(int(x * 1.5) for x in cap)
            self.cstep.close()
            self.cstep = None
            self.recaptures += 1
            self._capture(cams, idx, capacity=cap)
        return self.cstep.loss

    def step(self) -> torch.Tensor:
        """One iteration; returns the loss as a device scalar."""
        r, g = self.rast, self.g
        views = self._next_views()
        if self.captured:
            loss = self._captured_step(views)
            self.it += 1
            if (self.densify_from <= self.it < self.densify_until and self.densify_every > 0
                    and self.it % self.densify_every == 0):
                self.densify()
            return loss
        cams = [self.cams[v] for v in views]
        if self.partial:
            W, H = cams[0].width, cams[0].height
            keys = torch.randint(-2 ** 31, 2 ** 31, (W * H,), dtype=torch.int32, device=self.dev, generator=self.gen)
            off, pix = r.subsample(cams, keys)
            plane = torch.zeros((3, H, W), device=self.dev)
            _, fr = r.forward_partial(g, cams, off, pix, 0, images=[plane] * self.B)
            target = r.merge(fr, [self.targets[v] for v in views])
            loss, dl = r.loss_3d(fr, plane, target, self.w_l1, self.w_dssim)
            r.backward(g, fr, [dl] * self.B, densify=self.stats, grads=self.grads)
        else:
            imgs, fr = r.forward(g, cams)
            loss, dl = r.loss(cams, imgs, [self.targets[v] for v in views], self.w_l1, self.w_dssim)
            r.backward(g, fr, dl, densify=self.stats, grads=self.grads)
        r.release(fr)
        self.it += 1
        r.adam_step(g, self.grads, self.moments, self.it, self.lr)
        if (self.densify_from <= self.it < self.densify_until and self.densify_every > 0
                and self.it % self.densify_every == 0):
            self.densify()
        return loss

    def densify(self):
        """Multi-view adaptive density control now, from the statistics gathered since the last."""
        if self.cstep is not None:   # the captured step holds the old Gaussians
            torch.cuda.synchronize()
            self.cstep.close()
            self.cstep = None
        g = self.g
        normals = torch.randn((g.P, 2, 3), device=self.dev, generator=self.gen)
        adc = dict(self.adc)
        adc["min_opacity"] = adc["min_opacity"] * self.B
        new, src = self.rast.adapt_density(g, self.stats, normals, **adc)
        self.moments = self.rast.gather_rows(src, self.moments)
        self.g = new
        self.stats = _stats(new.P, self.dev)
        self.grads = _zeros_like_grads(new)
        self.n_densified += 1

    def run(self, n: int) -> List[float]:
        return [float(self.step().item()) for _ in range(n)]

    def close(self):
        if self.cstep is not None:
            self.cstep.close()
            self.cstep = None
        self.rast.close()


def _finish(sum_: torch.Tensor, acc: torch.Tensor, k: int) -> dict:
    a = acc.cpu().numpy()
    mean_sq = float(a[0]) / k
    sq_mean = float(a[1]) / (k * k)
    return dict(variance=mean_sq - sq_mean, mean_sq_norm=mean_sq, sq_norm_of_mean=sq_mean, batches=k)


def _moment_buffers(g: GaussianTensors):
    K = (g.sh_degree + 1) ** 2
    return (torch.zeros(g.P * (11 + 3 * K), dtype=torch.float64, device=g.means.device),
            torch.zeros(2, dtype=torch.float64, device=g.means.device))


def variance_views(rast: Rasterizer, g: GaussianTensors, cams, targets, batches, w_l1=1.0, w_dssim=0.0) -> dict:
    """Variance of the gradients of whole-view mini-batches: batch k renders the views batches[k]
    and takes the fused loss over them (the mean over their pixels)."""
    s, acc = _moment_buffers(g)
    grads = _zeros_like_grads(g)
    for views in batches:
        cb = [cams[v] for v in views]
        imgs, fr = rast.forward(g, cb)
        _, dl = rast.loss(cb, imgs, [targets[v] for v in views], w_l1, w_dssim)
        rast.backward(g, fr, dl, grads=grads)
        rast.release(fr)
        rast.grad_moments(g, grads, s, acc)
    return _finish(s, acc, len(batches))


def variance_partial(rast: Rasterizer, g: GaussianTensors, cams, targets, batches, keys, w_l1=1.0,
                     w_dssim=0.0) -> dict:
    """Variance of the gradients of partial-rendering mini-batches (Alg. 3): batch k shares the
    image plane among the views batches[k] by the sub-sampling keys keys[k] (int32 [H*W] on the
    GPU) and takes the L1 + 3D distance-aware D-SSIM loss over the merged plane."""
    s, acc = _moment_buffers(g)
    grads = _zeros_like_grads(g)
    for views, kk in zip(batches, keys):
        cb = [cams[v] for v in views]
        W, H = cb[0].width, cb[0].height
        off, pix = rast.subsample(cb, kk)
        plane = torch.zeros((3, H, W), device=g.means.device)
        _, fr = rast.forward_partial(g, cb, off, pix, 0, images=[plane] * len(cb))
        target = rast.merge(fr, [targets[v] for v in views])
        _, dl = rast.loss_3d(fr, plane, target, w_l1, w_dssim)
        rast.backward(g, fr, [dl] * len(cb), grads=grads)
        rast.release(fr)
        rast.grad_moments(g, grads, s, acc)
    return _finish(s, acc, len(batches))
