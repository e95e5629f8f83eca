"""Autotuner for the blend launch shape: tile size and pixels per lane.

Images, gradients and statistics do not depend on the tile shape or on how pixels map to lanes
(the footprint and the cut test decide coverage; tiles only bin work), so the choice is purely a
matter of speed. The tuner times a few forward + loss + backward steps of the caller's own batch
for each candidate and returns the fastest.
"""
from __future__ import annotations

import time
from typing import Iterable, List, Optional, Tuple

import torch

from .raster import GaussianTensors, Rasterizer

CANDIDATES: List[Tuple[Tuple[int, int], int]] = [
    ((16, 16), 2), ((16, 16), 4), ((32, 16), 4), ((16, 32), 4), ((32, 32), 4), ((32, 32), 2),
]


def time_config(g: GaussianTensors, cams, targets, tile, ppl, w_l1=1.0, w_dssim=0.0, steps=2, warmup=1) -> float:
    """Seconds per forward + loss + backward step with one launch shape."""
    r = Rasterizer(tile, ppl)
    try:
        def step():
            imgs, fr = r.forward(g, cams)
            _, dl = r.loss(cams, imgs, targets, w_l1, w_dssim)
            r.backward(g, fr, dl)
            r.release(fr)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps
    finally:
        r.close()


def autotune(g: GaussianTensors, cams, targets, w_l1=1.0, w_dssim=0.0,
             candidates: Optional[Iterable[Tuple[Tuple[int, int], int]]] = None, steps=2):
    """Returns ((tile_w, tile_h), pixels_per_lane, {candidate: seconds per step})."""
    cand = list(candidates or CANDIDATES)
    times = {}
    for tile, ppl in cand:
        times[(tile, ppl)] = time_config(g, cams, targets, tile, ppl, w_l1, w_dssim, steps=steps)
    best = min(times, key=times.get)
    return best[0], best[1], times
