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


def test_take_is_a_fifo_prefix_bounded_by_max_batch():
    adm = Admission(budget=1 << 40, n_slots=2, max_batch=3, bytes_per_pixel=10.0)
    q = _reqs([(10, 10)] * 7)
    b = adm.take(0, q)
    assert [r.rid for r in b] == [0, 1, 2]
    b2 = adm.take(1, q)
    assert [r.rid for r in b2] == [3, 4, 5]
    assert [r.rid for r in q] == [6]


def test_take_respects_the_budget_and_reserves():
    # 100 px per request: workspace 1.3 * 10 * px, image 12 * px
    adm = Admission(budget=5000, n_slots=2, max_batch=8, bytes_per_pixel=10.0, slack=1.3)
    q = _reqs([(10, 10)] * 5)
    b = adm.take(0, q)
    # k requests need 1300 k + 1200 k = 2500 k <= 5000 -> 2
    assert len(b) == 2
    assert adm.reserved[0] == 2600 and adm.images == 2400
    assert adm.used() <= adm.budget
    # nothing left for the other slot
    assert adm.take(1, q) == []
    adm.finish(0, b, held_after=2000, workspace=1500)
    assert adm.images == 0 and adm.reserved[0] == adm.held[0] == 2000
    # the estimate only grows: 1500 B over 200 px = 7.5 < 10
    assert adm.bpp == 10.0
    adm.finish(0, [], held_after=2000, workspace=None)


def test_refusal_raises_the_estimate_and_returns_images():
    adm = Admission(budget=10 ** 6, n_slots=1, max_batch=4, bytes_per_pixel=1.0, miss_growth=2.0)
    q = _reqs([(10, 10)] * 4)
    b = adm.take(0, q)
    assert len(b) == 4
    adm.refused(0, b, held_after=0)
    assert adm.images == 0 and adm.bpp == 2.0 and adm.misses == 1


def test_concurrent_refusals_raise_the_estimate_once():
    adm = Admission(budget=10 ** 6, n_slots=2, max_batch=2, bytes_per_pixel=1.0, miss_growth=2.0)
    q = _reqs([(10, 10)] * 4)
    b0, b1 = adm.take(0, q), adm.take(1, q)
    adm.refused(0, b0, 0)
    adm.refused(1, b1, 0)   # admitted under the same estimate: no second raise
    assert adm.bpp == 2.0 and adm.misses == 2
    q.extendleft(reversed(b1))
    q.extendleft(reversed(b0))
    b2 = adm.take(0, q)
    assert [r.rid for r in b2] == [0, 1]
    adm.refused(0, b2, 0)
    assert adm.bpp == 4.0


def test_fits_alone():
    adm = Admission(budget=10_000, n_slots=1, max_batch=4, bytes_per_pixel=10.0, slack=1.0)
    assert adm.fits_alone(Request(0, 0.0, _Cam(20, 20)))       # 4000 + 4800
    assert not adm.fits_alone(Request(0, 0.0, _Cam(30, 30)))   # 9000 + 10800


def test_budget_invariant_under_random_traffic():
    """A discrete simulation: random request sizes, random completion order, random exact
    workspaces within the library's limit. Used memory never exceeds the budget and every request
    is eventually served."""
    rng = np.random.default_rng(5)
    budget = 2_000_000
    adm = Admission(budget=budget, n_slots=3, max_batch=4, bytes_per_pixel=50.0)
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
            assert adm.fits_alone(q[0])
            adm.recycled(s)
            continue
        s = list(busy)[int(rng.integers(len(busy)))]
        b = busy.pop(s)
        pix = sum(r.pixels for r in b)
        limit = adm.reserved[s]
        need = int(adm.fixed + rng.uniform(20.0, 90.0) * pix)
        if max(adm.held[s], need) > limit:
            adm.refused(s, b, adm.held[s])
            q.extendleft(reversed(b))
        else:
            adm.finish(s, b, max(adm.held[s], need), need)
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


def test_per_view_bound_limits_batches_and_is_not_learned_per_pixel():
    # 100 px requests; per view 1000 B of records, 1 B/px; slack 1
    adm = Admission(budget=3000, n_slots=1, max_batch=8, view_bytes=1000, bytes_per_pixel=1.0, slack=1.0)
    q = _reqs([(10, 10)] * 4)
    b = adm.take(0, q)
    # k views need 1100 k + 1200 k (images) <= 3000 -> 1
    assert len(b) == 1 and adm.reserved[0] == 1100
    # a finished batch whose workspace is mostly records does not inflate the per-pixel estimate
    adm.finish(0, b, held_after=1050, workspace=1050)
    assert adm.bpp == 1.0
    adm.finish(0, [], held_after=1050, workspace=None)
    b = adm.take(0, q)
    adm.finish(0, b, held_after=1300, workspace=1300)
    assert adm.bpp == 3.0


def test_forced_admission_reserves_what_the_budget_has_left():
    adm = Admission(budget=10_000, n_slots=2, max_batch=4, bytes_per_pixel=100.0, slack=1.0)
    q = _reqs([(10, 10)])            # estimate 10,000 + 1,200 image bytes: over the budget
    assert adm.take(0, q) == []
    b = adm.take_forced(0, q)
    assert len(b) == 1 and not q
    assert adm.reserved[0] == 10_000 - 1_200 and adm.images == 1_200
    assert adm.used() <= adm.budget
    adm.refused(0, b, held_after=0)
    assert adm.used() == 0
