"""Render-request serving: a resident scene, continuous batching, HBM-budget admission.

Requests (one camera each) arrive over time. The server keeps the Gaussians on the GPU and runs
several worker slots; each slot is a library context with its own HIP stream and host thread.
An idle slot takes the next batch of waiting requests at once, so requests that arrive while
others are rendering are admitted as soon as a slot and memory are free, and the slots' batches
overlap on the device. Every view of a batch is rendered by one forward call (multi-view batch
of the multi-view appendix); a view's image does not depend on what else is in its batch.

Admission (class Admission) keeps the server's per-request device memory under a byte budget:
the memory every slot context holds plus the output images of requests in flight. As the
multi-view appendix sizes memory from the participating Gaussians before allocating, every queued
request gets its participation counts (records and covered tile pairs, mvgs_count_views, one
pre-pass over the waiting requests at a time), and a batch's memory is the exact bound the library
computes from them for the slot's context (mvgs_workspace_bound). A batch is the longest prefix of
the queue (in arrival order, at most `max_batch` views) whose bound and images fit in what the
budget leaves; the slot's context gets that bound as its workspace limit, which the library
enforces before it allocates, and which the forward then cannot exceed.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import _lib as L


@dataclass
class Request:
    rid: int
    arrival: float                  # seconds after the loop starts
    cam: object                     # scenes.Camera
    t_start: float = math.nan       # when its batch was launched
    t_done: float = math.nan        # when the host saw its batch complete
    slot: int = -1
    batch: int = -1
    image: Optional[object] = None  # [3,H,W] float32 on the GPU when images are kept
    error: Optional[str] = None
    records: int = -1               # participation pre-pass: participating Gaussians (-1: not counted)
    pairs: int = -1                 # and covered (Gaussian, tile) pairs

    @property
    def pixels(self) -> int:
        return int(self.cam.width) * int(self.cam.height)

    @property
    def image_bytes(self) -> int:
        return 12 * self.pixels


class Admission:
    """Byte accounting and batch formation against the budget (host logic only).

    bound(slot, reqs)  bytes slot `slot`'s context would hold after rendering `reqs` as one batch
    held[s]            bytes slot s's context holds (its buffers only grow until it is recycled)
    reserved[s]        what slot s may hold while it runs a batch (>= held[s]); == held[s] when idle
    images             bytes of output images of requests in flight
    """

    def __init__(self, budget: int, n_slots: int, max_batch: int, bound: Callable[[int, Sequence[Request]], int]):
        if budget <= 0 or n_slots < 1 or max_batch < 1:
            raise ValueError("budget, n_slots and max_batch must be positive")
        self.budget = int(budget)
        self.max_batch = int(max_batch)
        self.bound = bound
        self.held = [0] * n_slots
        self.reserved = [0] * n_slots
        self.images = 0
        self.peak = 0
        self.misses = 0

    def used(self) -> int:
        return sum(self.reserved) + self.images

    def take(self, slot: int, queue: deque) -> List[Request]:
        """Pop the longest admissible prefix of `queue` for an idle `slot` and reserve its memory.
        Returns [] when not even the head fits."""
        avail = self.budget - (self.used() - self.reserved[slot])
        n = img = 0
        need = 0
        items = list(queue)[:self.max_batch]
        for k in range(1, len(items) + 1):
            img_k = img + items[k - 1].image_bytes
            need_k = max(self.held[slot], int(self.bound(slot, items[:k])))
            if need_k + img_k > avail:
                break
            n, img, need = k, img_k, need_k
        if n == 0:
            return []
        batch = [queue.popleft() for _ in range(n)]
        self.reserved[slot] = need
        self.images += img
        self.peak = max(self.peak, self.used())
        return batch

    def finish(self, slot: int, batch: Sequence[Request], held_after: int):
        """The batch is done: its images leave the in-flight count (the caller owns them now) and the
        reservation falls back to what the context holds."""
        self.images -= sum(r.image_bytes for r in batch)
        self.held[slot] = self.reserved[slot] = int(held_after)

    def refused(self, slot: int, batch: Sequence[Request], held_after: int):
        """The library refused a batch under its reservation (the bound should make this never
        happen; counted)."""
        self.images -= sum(r.image_bytes for r in batch)
        self.held[slot] = self.reserved[slot] = int(held_after)
        self.misses += 1

    def recycled(self, slot: int):
        """The slot's context was destroyed and re-created empty."""
        self.held[slot] = self.reserved[slot] = 0


class _Slot:
    def __init__(self, server: "Server", index: int):
        import torch
        from .raster import Rasterizer
        self.server, self.index = server, index
        self.rast = Rasterizer(server.tile, server.ppl)
        self.stream = torch.cuda.Stream()          # default priority
        self.batch: Optional[List[Request]] = None
        self.limit = 0
        self.busy_intervals = []
        self.thread = threading.Thread(target=self._loop, name=f"mvgs-slot-{index}", daemon=True)
        self.thread.start()

    def recycle(self):
        from .raster import Rasterizer
        self.rast.close()
        self.rast = Rasterizer(self.server.tile, self.server.ppl)

    def _render(self, batch: List[Request], limit: int):
        import torch
        srv = self.server
        cams = [r.cam for r in batch]
        self.rast.set_workspace_limit(limit)
        with torch.cuda.stream(self.stream):
            imgs = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=srv.device) for c in cams]
            try:
                imgs, fr = self.rast.forward(srv.g, cams, imgs)
            except L.MvgsError as e:
                if e.status == L.MVGS_ECAPACITY:
                    return None
                raise
            self.rast.release(fr)   # the frame's buffers are reused only by later work on this stream
            ev = torch.cuda.Event()
            ev.record(self.stream)
        ev.synchronize()
        return imgs

    def _loop(self):
        srv = self.server
        while True:
            with srv.cond:
                while self.batch is None and not srv.stopping:
                    srv.cond.wait()
                if srv.stopping:
                    return
                batch, limit = self.batch, self.limit
            t0 = srv.clock()
            try:
                imgs = self._render(batch, limit)
                held = self.rast.memory_held()
                err = None
            except Exception as e:  # surfaced by Server.run
                imgs, held, err = None, 0, e
            t1 = srv.clock()
            with srv.cond:
                self.busy_intervals.append((t0, t1))
                if err is not None:
                    srv.error = err
                elif imgs is None:
                    srv.adm.refused(self.index, batch, held)
                    srv.queue.extendleft(reversed(batch))
                else:
                    srv.adm.finish(self.index, batch, held)
                    for r, im in zip(batch, imgs):
                        r.t_start, r.t_done, r.slot = t0, t1, self.index
                        r.image = im if srv.keep_images else None
                        srv.done.append(r)
                self.batch = None
                srv.cond.notify_all()


class Server:
    """Continuous-batching render server over a resident scene (GaussianTensors on the GPU)."""

    def __init__(self, g, n_slots: int = 4, budget_bytes: int = 16 << 30, max_batch: int = 8,
                 tile=(16, 16), pixels_per_lane: int = 0, keep_images: bool = False):
        import torch
        from .raster import Rasterizer
        g.check()
        self.g, self.device = g, g.means.device
        self.tile, self.ppl = tuple(tile), int(pixels_per_lane)
        self.keep_images = keep_images
        self.adm = Admission(budget_bytes, n_slots, max_batch, self._bound)
        # participation pre-pass of queued requests, on its own context and stream
        self.counter = Rasterizer(self.tile, self.ppl)
        self.count_stream = torch.cuda.Stream()    # default priority
        self.cond = threading.Condition()
        self.queue: deque = deque()
        self.done: List[Request] = []
        self.stopping = False
        self.error: Optional[BaseException] = None
        self.rejected: List[Request] = []
        self.batches = []          # (slot, number of views) per launched batch
        self.recycles = 0
        self._t0 = time.perf_counter()
        torch.cuda.synchronize()
        self.slots = [_Slot(self, i) for i in range(n_slots)]

    def clock(self) -> float:
        return time.perf_counter() - self._t0

    def close(self):
        with self.cond:
            self.stopping = True
            self.cond.notify_all()
        for s in self.slots:
            s.thread.join()
            s.rast.close()
        self.counter.close()

    def _bound(self, slot: int, reqs: Sequence[Request]) -> int:
        """Exact bytes slot `slot`'s context would hold after rendering `reqs` as one batch."""
        return self.slots[slot].rast.workspace_bound([r.cam for r in reqs], self.g.P, sum(r.records for r in reqs),
                                                     sum(r.pairs for r in reqs))

    def _count(self):
        """Participation counts of every queued request that has none (one pre-pass)."""
        import torch
        todo = [r for r in self.queue if r.records < 0]
        if not todo:
            return
        with torch.cuda.stream(self.count_stream):
            rec, pairs = self.counter.count_views(self.g, [r.cam for r in todo])
        for r, a, b in zip(todo, rec, pairs):
            r.records, r.pairs = int(a), int(b)

    def _idle(self):
        return [s for s in self.slots if s.batch is None]

    def _dispatch(self):
        self._count()
        while self.queue:
            idle = sorted(self._idle(), key=lambda s: -self.adm.held[s.index])
            if not idle:
                return
            launched = False
            for s in idle:
                batch = self.adm.take(s.index, self.queue)
                if batch:
                    self._launch(s, batch)
                    launched = True
                    break
            if launched:
                continue
            if len(idle) < len(self.slots):
                return   # wait for a busy slot to finish
            # every slot idle, yet the head does not fit: free idle contexts' memory; a request that
            # does not fit an empty context within the whole budget cannot be served
            big = idle[0]
            if self.adm.held[big.index] > 0:
                big.recycle()
                self.adm.recycled(big.index)
                self.recycles += 1
                continue
            r = self.queue.popleft()
            r.error = "request exceeds the memory budget"
            self.rejected.append(r)

    def _launch(self, s, batch):
        for r in batch:
            r.batch = len(self.batches)
        self.batches.append((s.index, len(batch)))
        s.batch, s.limit = batch, self.adm.reserved[s.index]
        self.cond.notify_all()

    def run(self, arrivals: Sequence[float], cams: Sequence, measure_from: int = 0) -> dict:
        """Serve requests arriving at `arrivals` (seconds from now, ascending). Returns statistics
        over requests with index >= measure_from."""
        reqs = [Request(i, float(a), c) for i, (a, c) in enumerate(zip(arrivals, cams))]
        pending = deque(reqs)
        self.batches = []
        self.adm.peak = self.adm.used()
        self.adm.misses = 0
        for s in self.slots:
            s.busy_intervals = []
        base = self.clock()
        for r in reqs:
            r.arrival += base
        with self.cond:
            while True:
                now = self.clock()
                while pending and pending[0].arrival <= now:
                    self.queue.append(pending.popleft())
                self._dispatch()
                if self.error is not None:
                    raise RuntimeError(f"serving slot failed: {self.error}") from self.error
                if not pending and not self.queue and len(self._idle()) == len(self.slots):
                    break
                timeout = max(0.0, pending[0].arrival - now) if pending else 0.5
                self.cond.wait(timeout)
        return self.stats(reqs, measure_from)

    def stats(self, reqs: Sequence[Request], measure_from: int = 0) -> dict:
        meas = [r for r in reqs[measure_from:] if r.error is None]
        lat = np.array([(r.t_done - r.arrival) * 1e3 for r in meas])
        if len(meas):
            window = max(r.t_done for r in meas) - min(r.arrival for r in meas)
        else:
            window = math.nan
        sizes = np.array([n for _, n in self.batches]) if self.batches else np.zeros(1)
        busy = [iv for s in self.slots for iv in s.busy_intervals]
        return {
            "requests": len(meas),
            "rejected": len([r for r in reqs[measure_from:] if r.error is not None]),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else math.nan,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else math.nan,
            "mean_ms": float(lat.mean()) if len(lat) else math.nan,
            "views_per_s": len(meas) / window if window > 0 else math.nan,
            "pixels_per_s": sum(r.pixels for r in meas) / window if window > 0 else math.nan,
            "mean_batch": float(sizes.mean()),
            "max_batch": int(sizes.max()),
            "overlap": overlap_fraction(busy),
            "peak_budget_bytes": int(self.adm.peak),
            "budget_bytes": int(self.adm.budget),
            "refused_batches": int(self.adm.misses),
            "recycled_slots": int(self.recycles),
        }


def overlap_fraction(intervals) -> float:
    """Fraction of the time some slot is busy during which at least two are."""
    ev = sorted([(a, 1) for a, b in intervals] + [(b, -1) for a, b in intervals])
    depth, last, any_t, two_t = 0, None, 0.0, 0.0
    for t, d in ev:
        if last is not None:
            if depth >= 1:
                any_t += t - last
            if depth >= 2:
                two_t += t - last
        depth += d
        last = t
    return two_t / any_t if any_t > 0 else 0.0
