"""Render-request serving: a resident scene, continuous batching, HBM-budget admission.

Requests (one camera each) arrive over time. The server keeps the Gaussians on the GPU and runs
several worker slots; each slot is a library context with its own HIP stream and host thread.
An idle slot takes the next batch of waiting requests at once, so requests that arrive while
others are rendering are admitted as soon as a slot and memory are free, and the slots' batches
overlap on the device. Every view of a batch is rendered by one forward call (multi-view batch
of the multi-view appendix); a view's image does not depend on what else is in its batch.

Admission (class Admission) keeps the server's per-request device memory under a byte budget:
the workspace every slot context holds plus the output images of requests in flight. A batch is
the longest prefix of the queue (in arrival order, at most `max_batch` views) whose estimated
workspace and images fit in what the budget leaves; the slot's context gets that reservation as
its workspace limit, which the library enforces before it allocates. A batch the library refuses
goes back to the head of the queue with a larger estimate. The per-pixel workspace estimate
learns from the exact workspace each finished batch reports.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass
from typing import List, Optional, Sequence

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

    @property
    def pixels(self) -> int:
        return int(self.cam.width) * int(self.cam.height)

    @property
    def image_bytes(self) -> int:
        return 12 * self.pixels


class Admission:
    """Byte accounting and batch formation against the budget (host logic only).

    held[s]      bytes slot s's context holds (its buffers only grow until the slot is recycled)
    reserved[s]  what slot s may hold while it runs a batch (>= held[s]); == held[s] when idle
    images       bytes of output images of requests in flight
    """

    def __init__(self, budget: int, n_slots: int, max_batch: int, fixed_bytes: int = 0, view_bytes: int = 0,
                 bytes_per_pixel: float = 256.0, slack: float = 1.3, miss_growth: float = 1.5):
        if budget <= 0 or n_slots < 1 or max_batch < 1:
            raise ValueError("budget, n_slots and max_batch must be positive")
        self.budget = int(budget)
        self.max_batch = int(max_batch)
        self.fixed = int(fixed_bytes)
        self.view_bytes = int(view_bytes)
        self.bpp = float(bytes_per_pixel)
        self.slack = float(slack)            # the context's allocator grows buffers with headroom
        self.miss_growth = float(miss_growth)
        self.held = [0] * n_slots
        self.reserved = [0] * n_slots
        self.images = 0
        self.peak = 0
        self.misses = 0
        self.gen = 0                        # bumped whenever the estimate is raised after a refusal
        self.taken_gen = [0] * n_slots      # estimate generation each slot's batch was admitted with

    def used(self) -> int:
        return sum(self.reserved) + self.images

    def workspace_estimate(self, views: int, pixels: int) -> int:
        """Workspace of a batch: a part per batch, a bound per view (records, one per Gaussian that
        takes part, at most P) and a learned part per pixel (pairs and per-pixel blend state)."""
        return int(self.fixed + self.view_bytes * views + self.bpp * pixels)

    def _need(self, slot: int, views: int, pixels: int, image_bytes: int) -> int:
        return max(self.held[slot], int(self.slack * self.workspace_estimate(views, pixels))) + image_bytes

    def fits_alone(self, req: Request) -> bool:
        """Whether the request could run with every other slot empty."""
        return int(self.slack * self.workspace_estimate(1, req.pixels)) + req.image_bytes <= self.budget

    def take(self, slot: int, queue: deque) -> List[Request]:
        """Pop the longest admissible prefix of `queue` for an idle `slot` and reserve its memory.
        Returns [] when not even the head fits."""
        avail = self.budget - (self.used() - self.reserved[slot])
        n = pix = img = 0
        for r in queue:
            if n == self.max_batch or self._need(slot, n + 1, pix + r.pixels, img + r.image_bytes) > avail:
                break
            n += 1
            pix += r.pixels
            img += r.image_bytes
        if n == 0:
            return []
        batch = [queue.popleft() for _ in range(n)]
        self.taken_gen[slot] = self.gen
        self.reserved[slot] = max(self.held[slot], int(self.slack * self.workspace_estimate(n, pix)))
        self.images += img
        self.peak = max(self.peak, self.used())
        return batch

    def take_forced(self, slot: int, queue: deque) -> List[Request]:
        """The head alone, reserving everything the budget has left (used when every slot is idle
        and holds nothing, yet the estimate says the head does not fit: the library decides)."""
        r = queue.popleft()
        self.taken_gen[slot] = self.gen
        self.reserved[slot] = max(self.held[slot], self.budget - (self.used() - self.reserved[slot]) - r.image_bytes)
        self.images += r.image_bytes
        self.peak = max(self.peak, self.used())
        return [r]

    def finish(self, slot: int, batch: Sequence[Request], held_after: int, workspace: Optional[int]):
        """The batch is done: its images leave the in-flight count (the caller owns them now), the
        reservation falls back to what the context holds, and the estimate learns."""
        self.images -= sum(r.image_bytes for r in batch)
        self.held[slot] = self.reserved[slot] = int(held_after)
        pix = sum(r.pixels for r in batch)
        if workspace is not None and pix > 0:
            self.bpp = max(self.bpp, (workspace - self.fixed - self.view_bytes * len(batch)) / pix)

    def refused(self, slot: int, batch: Sequence[Request], held_after: int):
        """The library refused the batch under its reservation: release, and estimate higher unless
        the estimate was already raised since this batch was admitted."""
        self.images -= sum(r.image_bytes for r in batch)
        self.held[slot] = self.reserved[slot] = int(held_after)
        if self.taken_gen[slot] == self.gen:
            self.bpp *= self.miss_growth
            self.gen += 1
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
        self.forced = False   # the batch was admitted with the whole remaining budget
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
                    return None, None
                raise
            ws = fr.workspace()
            self.rast.release(fr)   # the frame's buffers are reused only by later work on this stream
            ev = torch.cuda.Event()
            ev.record(self.stream)
        ev.synchronize()
        return imgs, ws

    def _loop(self):
        srv = self.server
        while True:
            with srv.cond:
                while self.batch is None and not srv.stopping:
                    srv.cond.wait()
                if srv.stopping:
                    return
                batch, limit, forced = self.batch, self.limit, self.forced
            t0 = srv.clock()
            try:
                imgs, ws = self._render(batch, limit)
                held = self.rast.memory_held()
                err = None
            except Exception as e:  # surfaced by Server.run
                imgs, ws, held, err = None, None, 0, e
            t1 = srv.clock()
            with srv.cond:
                self.busy_intervals.append((t0, t1))
                if err is not None:
                    srv.error = err
                elif imgs is None:
                    srv.adm.refused(self.index, batch, held)
                    if forced:
                        # refused with every byte the budget has: the request cannot be served
                        for r in batch:
                            r.error = "request exceeds the memory budget"
                            srv.rejected.append(r)
                    else:
                        srv.queue.extendleft(reversed(batch))
                else:
                    srv.adm.finish(self.index, batch, held, ws)
                    for r, im in zip(batch, imgs):
                        r.t_start, r.t_done, r.slot = t0, t1, self.index
                        r.image = im if srv.keep_images else None
                        srv.done.append(r)
                self.batch = None
                srv.cond.notify_all()


# Device bytes per participating (view, Gaussian) record in a forward: the 64-byte blend record, its
# view (2), depth keys and record indices double-buffered (16), tile rectangle in record and in depth
# order (32), pair count and offset (8).
RECORD_BYTES = 122


class Server:
    """Continuous-batching render server over a resident scene (GaussianTensors on the GPU)."""

    def __init__(self, g, n_slots: int = 4, budget_bytes: int = 16 << 30, max_batch: int = 8,
                 tile=(16, 16), pixels_per_lane: int = 0, keep_images: bool = False,
                 bytes_per_pixel: float = 64.0):
        import torch
        g.check()
        self.g, self.device = g, g.means.device
        self.tile, self.ppl = tuple(tile), int(pixels_per_lane)
        self.keep_images = keep_images
        # per batch: Gaussian-sized counters and offsets, upload staging, page rounding; per view: at
        # most P records of RECORD_BYTES each
        self.adm = Admission(budget_bytes, n_slots, max_batch, fixed_bytes=16 * (g.P + 1) + (256 << 10),
                             view_bytes=RECORD_BYTES * g.P, bytes_per_pixel=bytes_per_pixel)
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

    def _idle(self):
        return [s for s in self.slots if s.batch is None]

    def _dispatch(self):
        while self.queue:
            idle = sorted(self._idle(), key=lambda s: -self.adm.held[s.index])
            if not idle:
                return
            launched = False
            for s in idle:
                batch = self.adm.take(s.index, self.queue)
                if batch:
                    self._launch(s, batch, forced=False)
                    launched = True
                    break
            if launched:
                continue
            if len(idle) < len(self.slots):
                return   # wait for a busy slot to finish
            # every slot idle, yet the head does not fit the estimate: free idle contexts' memory,
            # then let the library decide with the whole budget
            big = idle[0]
            if self.adm.held[big.index] > 0:
                big.recycle()
                self.adm.recycled(big.index)
                self.recycles += 1
                continue
            self._launch(big, self.adm.take_forced(big.index, self.queue), forced=True)

    def _launch(self, s, batch, forced):
        for r in batch:
            r.batch = len(self.batches)
        self.batches.append((s.index, len(batch)))
        s.batch, s.limit, s.forced = batch, self.adm.reserved[s.index], forced
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
