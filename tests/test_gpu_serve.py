"""The serving loop on the GPU: every request's image, rendered inside a batch of whatever arrived
with it and while other slots render, equals the same view rendered alone, bit for bit; the HBM
budget holds; slots overlap."""
import math

import pytest
import torch

from paper_2506_12727_amd import scenes
from paper_2506_12727_amd.raster import GaussianTensors, Rasterizer
from paper_2506_12727_amd.serve import Server

from gpu_common import needs_gpu

pytestmark = pytest.mark.gpu

RES = [(64, 64), (160, 120), (320, 180), (96, 200)]


def _alone_equal(g, reqs, tile):
    r = Rasterizer(tile)
    try:
        for q in reqs:
            assert q.error is None, q.error
            im, fr = r.forward(g, [q.cam])
            r.release(fr)
            assert torch.equal(im[0], q.image), q.rid
    finally:
        r.close()


def test_serving_results_equal_alone_renders():
    needs_gpu()
    sc = scenes.make_scene(20000, 3, log_scale_mean=-3.5)
    g = GaussianTensors.from_scene(sc)
    arr, cams = scenes.make_requests(48, rate_hz=20000.0, resolutions=RES)
    srv = Server(g, n_slots=2, budget_bytes=1 << 30, max_batch=4, keep_images=True)
    try:
        st = srv.run(arr, cams)
        reqs = sorted(srv.done, key=lambda r: r.rid)
    finally:
        srv.close()
    assert st["requests"] == 48 and st["rejected"] == 0
    assert st["max_batch"] >= 2, st
    assert len({r.slot for r in reqs}) == 2
    assert st["peak_budget_bytes"] <= st["budget_bytes"]
    assert all(r.t_done >= r.arrival for r in reqs)
    _alone_equal(g, reqs, (16, 16))


def test_serving_under_a_tight_budget():
    """A budget that admits about two requests at a time and an estimate that starts far too low:
    the library refuses batches, they return to the queue, and every result is still exact."""
    needs_gpu()
    sc = scenes.make_scene(20000, 3, log_scale_mean=-3.5)
    g = GaussianTensors.from_scene(sc)
    arr, cams = scenes.make_requests(24, rate_hz=math.inf, resolutions=RES)
    # workspace of the largest request alone
    r = Rasterizer((16, 16))
    big = max(cams, key=lambda c: c.width * c.height)
    _, fr = r.forward(g, [big])
    ws = fr.workspace()
    r.release(fr)
    r.close()
    budget = int(4 * ws)
    srv = Server(g, n_slots=2, budget_bytes=budget, max_batch=4, keep_images=True, bytes_per_pixel=1.0)
    try:
        st = srv.run(arr, cams)
        reqs = sorted(srv.done, key=lambda q: q.rid)
        held = sum(s.rast.memory_held() for s in srv.slots)
    finally:
        srv.close()
    assert st["requests"] == 24 and st["rejected"] == 0, st
    assert st["refused_batches"] >= 1
    assert st["peak_budget_bytes"] <= budget
    assert held <= budget
    _alone_equal(g, reqs, (16, 16))
