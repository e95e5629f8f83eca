"""A training step captured into a HIP graph.

The step (forward over a batch of views, fused loss, backward with optional densification
statistics) runs in capacity mode, where the library's forward needs no host synchronization, so
the whole step is one graph: a replay launches every kernel of the step with no host work between
them. The graph keeps its tensors: write new targets into `targets` before a replay, and change the
batch's poses with `set_cameras` (same image sizes). Each replay overwrites `images`, `loss`,
`dl` and `grads` and adds to the statistics. `check()` waits and raises if the last replay's
records or pairs exceeded the capacities (its results are then void).

With `partial=True` the step is the thread-efficient partial rendering of Alg. 3: the views (of
one size) share one image plane by the per-position keys in `keys` (int32 [H*W]; each replay
draws new ones into it first unless `fresh_keys=False`, then the caller writes them), the
targets are merged into `target_plane` by the same selection, and the loss is L1 + the 3D
distance-aware D-SSIM of Sec. 5.1.2 on the plane (`plane`, its gradient `dl_plane`).

With `optimizer` = dict(moments, lr, step[, beta1, beta2, eps]) the step ends with the Adam update
of the Gaussians, its step number counted on the device in `step` (int32 [1]), and skipped when
the forward overflowed its capacities. The warm-up call that sizes the buffers is then a full
training step too.
"""
from __future__ import annotations

import math
from typing import Optional

import torch

from .raster import GaussianTensors, Rasterizer


def measure_capacity(g: GaussianTensors, cams, tile=(16, 16), ppl=0, headroom: float = 1.25):
    """Records and pairs of one eager forward of this batch, times `headroom`."""
    r = Rasterizer(tile, ppl)
    try:
        _, fr = r.forward(g, cams)
        info = fr.info()
        r.release(fr)
    finally:
        r.close()
    return (max(1, int(math.ceil(info["records"] * headroom))), max(1, int(math.ceil(info["pairs"] * headroom))))


def measure_capacity_pool(g: GaussianTensors, cams, views_per_batch: int, tile=(16, 16), ppl=0,
                          headroom: float = 1.25):
    """Capacities that hold any batch of `views_per_batch` views of the pool `cams`: the records
    and pairs of each view rendered alone, the largest ones summed, times `headroom`."""
    r = Rasterizer(tile, ppl)
    recs, pairs = [], []
    try:
        for c in cams:
            _, fr = r.forward(g, [c])
            info = fr.info()
            r.release(fr)
            recs.append(info["records"])
            pairs.append(info["pairs"])
    finally:
        r.close()
    top = lambda xs: sum(sorted(xs, reverse=True)[:views_per_batch])
    return (max(1, int(math.ceil(top(recs) * headroom))), max(1, int(math.ceil(top(pairs) * headroom))))


class CapturedStep:
    def __init__(self, g: GaussianTensors, cams, targets, w_l1=1.0, w_dssim=0.0, tile=(16, 16), ppl=0,
                 capacity=None, densify: Optional[dict] = None, partial: bool = False, fresh_keys: bool = True,
                 optimizer: Optional[dict] = None):
        g.check()
        self.g, self.cams = g, list(cams)
        self.w_l1, self.w_dssim = float(w_l1), float(w_dssim)
        self.partial, self.fresh_keys = bool(partial), bool(fresh_keys)
        if self.partial and len({(c.width, c.height) for c in self.cams}) != 1:
            raise ValueError("partial rendering shares one image plane: the views must have one size")
        if capacity is None:
            capacity = measure_capacity(g, cams, tile, ppl)
        self.rast = Rasterizer(tile, ppl, capacity=capacity)
        dev = g.means.device
        self.targets = [t.contiguous() for t in targets]
        if self.partial:
            W, H = self.cams[0].width, self.cams[0].height
            self.keys = torch.randint(-2 ** 31, 2 ** 31, (W * H,), dtype=torch.int32, device=dev)
            self.plane = torch.zeros((3, H, W), device=dev)
            self.target_plane = torch.zeros((3, H, W), device=dev)
            self.dl_plane = torch.empty((3, H, W), device=dev)
            self.images = [self.plane] * len(self.cams)
            self.dl = [self.dl_plane] * len(self.cams)
        else:
            self.images = [torch.empty((3, c.height, c.width), device=dev) for c in cams]
            self.dl = [torch.empty_like(t) for t in self.images]
        self.loss = torch.empty(1, device=dev)
        self.grads = dict(means=torch.empty_like(g.means), scales=torch.empty_like(g.scales),
                          quats=torch.empty_like(g.quats), opacities=torch.empty_like(g.opacities),
                          sh=torch.empty_like(g.sh))
        self.densify = densify
        self.optimizer = optimizer
        if optimizer is not None:
            st = optimizer["step"]
            if st.dtype != torch.int32 or st.numel() != 1 or not st.is_cuda:
                raise ValueError("optimizer['step'] must be an int32 [1] tensor on the GPU")
        # one step outside the capture sizes every buffer; its frame returns to the pool
        fr = self._step()
        fr.check()
        self.rast.release(fr)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.frame = self._step()
        torch.cuda.synchronize()

    def _step(self):
        r = self.rast
        if self.partial:
            if self.fresh_keys:
                self.keys.random_(-2 ** 31, 2 ** 31)
            off, pix = r.subsample(self.cams, self.keys)
            _, fr = r.forward_partial(self.g, self.cams, off, pix, 0, images=self.images)
            r.merge(fr, self.targets, out=self.target_plane)
            r.loss_3d(fr, self.plane, self.target_plane, self.w_l1, self.w_dssim, out=self.loss, grad=self.dl_plane)
        else:
            _, fr = r.forward(self.g, self.cams, images=self.images)
            r.loss(self.cams, self.images, self.targets, self.w_l1, self.w_dssim, out=self.loss, grads=self.dl)
        r.backward(self.g, fr, self.dl, densify=self.densify, grads=self.grads)
        if self.optimizer is not None:
            o = self.optimizer
            r.adam_step(self.g, self.grads, o["moments"], 0, o["lr"], o.get("beta1", 0.9), o.get("beta2", 0.999),
                        o.get("eps", 1e-15), step_dev=o["step"], skip=fr)
        return fr

    def replay(self):
        self.graph.replay()

    def set_cameras(self, cams):
        """New poses for the next replays (same sizes). No replay may be in flight."""
        self.frame.set_cameras(cams)
        self.cams = list(cams)

    def check(self):
        self.frame.check()

    def close(self):
        self.graph = None
        if self.frame is not None:
            self.rast.release(self.frame)
            self.frame = None
        self.rast.close()
