"""Autotuner for the blend launch shape: tile size and pixels per lane.

Images, gradients and statistics do not depend on the tile shape or on how pixels map to lanes
(the footprint and the cut test decide coverage; tiles only bin work), so the choice is purely a
matter of speed. The tuner times forward + loss + backward steps of the caller's own batch for
each candidate in two rounds: every candidate for a few steps, then the fastest few again for more
steps; a candidate's time is the median of its per-step times (one synchronisation per step), so
one slow step does not decide. Results are kept in a JSON file keyed by the device and the batch
(Gaussian count, SH degree, view sizes, loss), so a later run on the same kind of batch reuses them.
"""
from __future__ import annotations

import json
import os
import statistics
import time
from typing import Dict, Iterable, List, Optional, Tuple

import torch

from .raster import GaussianTensors, Rasterizer

# one pixel per lane (more wavefronts per tile) wins on small frames, whose few tiles leave
# most of the chip idle at 2 or 4
CANDIDATES: List[Tuple[Tuple[int, int], int]] = [
    ((16, 16), 2), ((16, 16), 4), ((32, 16), 4), ((16, 32), 4), ((32, 32), 4), ((32, 32), 2),
    ((32, 16), 2), ((16, 32), 2), ((16, 16), 1), ((8, 8), 1),
]

CACHE_ENV = "MVGS_TUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(os.path.expanduser("~"), ".cache", "mvgs", "tune.json")


def batch_key(g: GaussianTensors, cams, w_l1: float, w_dssim: float) -> str:
    """What the best launch shape depends on: the device, the scene size and the batch's views."""
    dev = torch.cuda.get_device_name(g.means.device) if g.means.is_cuda else "cpu"
    sizes = ",".join(f"{c.width}x{c.height}" for c in cams)
    return f"{dev}|P={g.P}|sh={g.sh_degree}|views={sizes}|l1={w_l1:g}|dssim={w_dssim:g}"


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, entry: dict) -> None:
    d = _load(path)
    d[key] = entry
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = f"{path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass   # a cache that cannot be written only costs the next run a tuning pass


def step_times(g: GaussianTensors, cams, targets, tile, ppl, w_l1=1.0, w_dssim=0.0, steps=3,
               warmup=1) -> List[float]:
    """Seconds of each of `steps` forward + loss + backward steps with one launch shape."""
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
        out = []
        for _ in range(steps):
            t0 = time.perf_counter()
            step()
            torch.cuda.synchronize()
            out.append(time.perf_counter() - t0)
        return out
    finally:
        r.close()


def time_config(g: GaussianTensors, cams, targets, tile, ppl, w_l1=1.0, w_dssim=0.0, steps=3, warmup=1) -> float:
    """Median seconds per forward + loss + backward step with one launch shape."""
    return statistics.median(step_times(g, cams, targets, tile, ppl, w_l1, w_dssim, steps, warmup))


def autotune(g: GaussianTensors, cams, targets, w_l1=1.0, w_dssim=0.0,
             candidates: Optional[Iterable[Tuple[Tuple[int, int], int]]] = None, steps=3, finalists=3,
             final_steps=8, cache: bool = True):
    """Returns ((tile_w, tile_h), pixels_per_lane, {candidate: median seconds per step}). With
    `cache`, a result stored for the same device and batch is returned without timing, and a new
    one is stored."""
    cand = list(candidates or CANDIDATES)
    key = batch_key(g, cams, w_l1, w_dssim)
    path = cache_path()
    if cache:
        hit = _load(path).get(key)
        if hit and [list(t) + [p] for t, p in cand] == hit.get("candidates"):
            times = {(tuple(t), p): s for t, p, s in hit["times"]}
            return tuple(hit["tile"]), int(hit["ppl"]), times
    times = {c: time_config(g, cams, targets, c[0], c[1], w_l1, w_dssim, steps=steps) for c in cand}
    for c in sorted(times, key=times.get)[:max(1, finalists)]:
        times[c] = time_config(g, cams, targets, c[0], c[1], w_l1, w_dssim, steps=final_steps)
    best = min(times, key=times.get)
    if cache:
        _store(path, key, {"tile": list(best[0]), "ppl": best[1],
                           "candidates": [list(t) + [p] for t, p in cand],
                           "times": [[list(t), p, s] for (t, p), s in times.items()]})
    return best[0], best[1], times
