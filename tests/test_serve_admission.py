"""Host logic of the serving loop: batch formation and HBM-budget accounting (no GPU)."""
import math
from collections import deque

import numpy as np
import pytest

from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.serve import Admission, Request, overlap_fraction


class _Cam:
    def __init__(self, w, h):
        self.width, self.height = w, h


def _reqs(sizes):
    return deque(Request(i, 0.0, _Cam(w, h)) for i, (w, h) in enumerate(sizes))


def _linear_bound(adm, fixed=0, per_view=0, per_pixel=10):
    """A stand-in for the library's exact bound: what the slot holds grows to fixed + per view +
    per pixel of the batch."""
    return lambda slot, reqs: max(adm.held[slot], fixed + per_view * len(reqs) + per_pixel * sum(r.pixels for r in reqs))


def _adm(budget, n_slots, max_batch, **kw):
    adm = Admission(budget=budget, n_slots=n_slots, max_batch=max_batch, bound=lambda s, r: 0)
    adm.bound = _linear_bound(adm, **kw)
    return adm


def test_take_is_a_fifo_prefix_bounded_by_max_batch():
    adm = _adm(1 << 40, 2, 3)
    q = _reqs([(10, 10)] * 7)
    b = adm.take(0, q)
    assert [r.rid for r in b] == [0, 1, 2]
    b2 = adm.take(1, q)
    assert [r.rid for r in b2] == [3, 4, 5]
    assert [r.rid for r in q] == [6]


def test_take_respects_the_budget_and_reserves_the_bound():
    # 100 px per request: bound 10 B/px, images 12 B/px
    adm = _adm(5000, 2, 8)
    q = _reqs([(10, 10)] * 5)
    b = adm.take(0, q)
    # k requests need 1000 k + 1200 k <= 5000 -> 2
    assert len(b) == 2
    assert adm.reserved[0] == 2000 and adm.images == 2400
    assert adm.used() <= adm.budget
    # nothing left for the other slot
    assert adm.take(1, q) == []
    adm.finish(0, b, held_after=2000)
    assert adm.images == 0 and adm.reserved[0] == adm.held[0] == 2000


def test_bound_is_asked_per_prefix_for_the_slot():
    seen = []

    def bound(slot, reqs):
        seen.append((slot, [r.rid for r in reqs]))
        return 100 * len(reqs)

    adm = Admission(budget=10 ** 6, n_slots=2, max_batch=3, bound=bound)
    q = _reqs([(10, 10)] * 5)
    adm.take(1, q)
    assert seen == [(1, [0]), (1, [0, 1]), (1, [0, 1, 2])]
    assert adm.reserved[1] == 300


def test_refusal_returns_images_and_counts():
    adm = _adm(10 ** 6, 1, 4)
    q = _reqs([(10, 10)] * 4)
    b = adm.take(0, q)
    assert len(b) == 4
    adm.refused(0, b, held_after=0)
    assert adm.images == 0 and adm.misses == 1 and adm.used() == 0


def test_budget_invariant_under_random_traffic():
    """A discrete simulation: random request sizes, random completion order; each finished batch
    leaves its slot holding the bound it was admitted with (the library's exact bound). Used memory
    never exceeds the budget and every request that fits an empty slot is served."""
    rng = np.random.default_rng(5)
    budget = 2_000_000
    adm = _adm(budget, 3, 4, fixed=20_000, per_view=5_000, per_pixel=50)
    sizes = [(int(rng.integers(8, 120)), int(rng.integers(8, 120))) for _ in range(300)]
    q = _reqs(sizes)
    busy = {}
    served = 0
    while q or busy:
        for s in range(3):
            if s not in busy and q:
                b = adm.take(s, q)
                if b:
                    busy[s] = b
                assert adm.used() <= budget
        if not busy:
            # every slot idle and the head does not fit: recycle the largest
            s = int(np.argmax(adm.held))
            assert adm.held[s] > 0
            adm.recycled(s)
            continue
        s = list(busy)[int(rng.integers(len(busy)))]
        b = busy.pop(s)
        adm.finish(s, b, adm.reserved[s])
        served += len(b)
        assert adm.used() <= budget
    assert served == len(sizes)
    assert adm.peak <= budget


def test_overlap_fraction():
    assert overlap_fraction([]) == 0.0
    assert overlap_fraction([(0, 1), (2, 3)]) == 0.0
    assert math.isclose(overlap_fraction([(0, 2), (1, 3)]), 1 / 3)
    assert math.isclose(overlap_fraction([(0, 4), (0, 4)]), 1.0)


def test_request_stream_is_seeded_poisson():
    arr, cams = scenes.make_requests(4000, rate_hz=200.0)
    arr2, cams2 = scenes.make_requests(4000, rate_hz=200.0)
    assert np.array_equal(arr, arr2)
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert np.all(gaps > 0)
    # exponential gaps with mean 5 ms: mean within 5 %, coefficient of variation near 1
    assert abs(gaps.mean() - 0.005) < 0.00025
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05
    res = {(c.width, c.height) for c in cams}
    assert res == set(scenes.SERVE_RESOLUTIONS)
    for c in cams[:50]:
        pos = -c.R.T.astype(np.float64) @ c.t.astype(np.float64)
        assert abs(np.linalg.norm(pos) - 3.0) < 1e-4
    a0, _ = scenes.make_requests(10, rate_hz=math.inf)
    assert np.all(a0 == 0.0)
