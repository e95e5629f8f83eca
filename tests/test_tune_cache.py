"""Autotuner bookkeeping on the CPU: the persisted results are keyed by device and batch, reused
without timing, and a cache for another candidate list is not trusted."""
import json

import numpy as np
import pytest
import torch

from paper_2506_12727_amd import scenes, tune
from paper_2506_12727_amd.raster import GaussianTensors


def _batch():
    sc = scenes.make_scene(100, 0)
    g = GaussianTensors.from_scene(sc, device="cpu")
    cams = scenes.make_cameras([(64, 48), (32, 32)])
    return g, cams


def test_cached_result_is_reused_without_timing(tmp_path, monkeypatch):
    monkeypatch.setenv(tune.CACHE_ENV, str(tmp_path / "tune.json"))
    g, cams = _batch()
    calls = []

    def fake(g_, cams_, tg, tile, ppl, w_l1, w_dssim, steps=3, warmup=1):
        calls.append((tile, ppl, steps))
        return {((32, 32), 4): 1.0, ((16, 16), 2): 2.0}.get((tile, ppl), 3.0) + 0.001 * steps

    monkeypatch.setattr(tune, "time_config", fake)
    tile, ppl, times = tune.autotune(g, cams, None)
    assert (tile, ppl) == ((32, 32), 4)
    n_first = len(calls)
    # every candidate once, then the three fastest again with more steps
    assert n_first == len(tune.CANDIDATES) + 3
    assert sum(1 for c in calls if c[2] == 8) == 3
    tile2, ppl2, times2 = tune.autotune(g, cams, None)
    assert (tile2, ppl2) == (tile, ppl) and len(calls) == n_first
    assert times2 == times
    d = json.load(open(tmp_path / "tune.json"))
    assert list(d) == [tune.batch_key(g, cams, 1.0, 0.0)]
    # another batch, another key
    tune.autotune(g, cams[:1], None)
    assert len(calls) > n_first
    assert len(json.load(open(tmp_path / "tune.json"))) == 2


def test_cache_for_other_candidates_is_not_used(tmp_path, monkeypatch):
    monkeypatch.setenv(tune.CACHE_ENV, str(tmp_path / "tune.json"))
    g, cams = _batch()
    monkeypatch.setattr(tune, "time_config", lambda *a, **k: 1.0 if a[3] == (16, 16) and a[4] == 2 else 2.0)
    tune.autotune(g, cams, None, candidates=[((16, 16), 2), ((32, 32), 4)])
    seen = []
    monkeypatch.setattr(tune, "time_config", lambda *a, **k: seen.append(a[3:5]) or 1.0)
    tune.autotune(g, cams, None, candidates=[((32, 32), 4)])
    assert seen   # the stored entry was for a different candidate list: timed again


def test_unwritable_cache_is_harmless(tmp_path, monkeypatch):
    blocker = tmp_path / "file"
    blocker.write_text("x")
    monkeypatch.setenv(tune.CACHE_ENV, str(blocker / "sub" / "tune.json"))
    g, cams = _batch()
    monkeypatch.setattr(tune, "time_config", lambda *a, **k: 1.0)
    assert tune.autotune(g, cams, None)[0] in [c[0] for c in tune.CANDIDATES]
