"""The oracle's pixel sub-sampling for thread-efficient partial rendering (Alg. 3), pinned by a
hand-worked fixture and by invariants; and the two facts the partial path rests on: a pixel's
value does not depend on which other pixels are rendered, and the backward is linear in dL/dimage,
so rendering a selection is the full render restricted to it."""
import json
import os

import numpy as np

import oracle
from paper_2506_12727_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "partition_4x2_three_views.json")


def test_partition_hand_worked_fixture():
    f = json.load(open(GOLDEN))
    off, pix = oracle.subsample_tiles(f["width"], f["height"], f["views"], f["tile"], f["keys"])
    segs = [list(pix[off[s]:off[s + 1]]) for s in range(len(off) - 1)]
    assert segs == f["segments_in_position_order"]
    # the ranking itself: rank r goes to view r mod 3
    for r, p in enumerate(f["ranked_positions"]):
        assert p in segs[r % 3]


def _check_partition(W, H, B, tile, keys):
    off, pix = oracle.subsample_tiles(W, H, B, tile, keys)
    tw, th = tile
    txn, tyn = (W + tw - 1) // tw, (H + th - 1) // th
    T = txn * tyn
    assert len(off) == B * T + 1 and off[0] == 0 and off[-1] == W * H == len(pix)
    # every position exactly once over all views
    assert np.array_equal(np.sort(pix), np.arange(W * H))
    k = np.asarray(keys, np.uint32).reshape(-1)
    for t in range(T):
        tx, ty = t % txn, t // txn
        n = (min(W, tx * tw + tw) - tx * tw) * (min(H, ty * th + th) - ty * th)
        ranked = []
        for v in range(B):
            seg = pix[off[v * T + t]:off[v * T + t + 1]]
            # balanced: view v gets the ranks v, v + B, v + 2B, ...
            assert len(seg) == max(0, -(-(n - v) // B))
            assert np.all(np.diff(seg.astype(np.int64)) > 0)   # ascending position
            xs, ys = seg % W, seg // W
            assert np.all(xs // tw == tx) and np.all(ys // th == ty)
            # in (key, position) order, the segment's pixels are the ranks v, v + B, ...
            ranked.append(sorted(seg.tolist(), key=lambda p: (int(k[p]), p)))
        # interleaving the views' ranked pixels gives the tile's positions in (key, position) order
        order = [ranked[r % B][r // B] for r in range(n)]
        kk = [(int(k[p]), int(p)) for p in order]
        assert kk == sorted(kk)
    return off, pix


def test_partition_invariants_ragged():
    rng = np.random.default_rng(0)
    for (W, H, B, tile) in [(37, 29, 3, (16, 16)), (33, 17, 4, (8, 8)), (20, 40, 5, (32, 16)), (9, 7, 1, (8, 8))]:
        keys = rng.integers(0, 2 ** 32, size=W * H, dtype=np.uint64).astype(np.uint32)
        _check_partition(W, H, B, tile, keys)
    # heavy ties: the position index decides
    keys = rng.integers(0, 3, size=37 * 29).astype(np.uint32)
    _check_partition(37, 29, 3, (16, 16), keys)


def test_more_views_than_pixels_in_a_tile():
    keys = np.arange(6, dtype=np.uint32)[::-1].copy()
    off, pix = _check_partition(3, 2, 8, (8, 8), keys)
    # six pixels, eight views: views 6 and 7 get nothing; the keys fall with position, so view v
    # gets the position of rank v, 5 - v
    assert [len(pix[off[v]:off[v + 1]]) for v in range(8)] == [1, 1, 1, 1, 1, 1, 0, 0]
    assert list(pix) == [5, 4, 3, 2, 1, 0]


def test_selection_renders_as_the_full_image_and_backward_is_linear():
    sc = scenes.make_scene(400, 2, log_scale_mean=-2.6)
    cams = scenes.make_cameras([(40, 24), (40, 24)])
    full = oracle.forward(sc, cams, (8, 8))
    keys = np.random.default_rng(4).integers(0, 2 ** 32, size=40 * 24, dtype=np.uint64).astype(np.uint32)
    off, pix = oracle.subsample_tiles(40, 24, 2, (8, 8), keys)
    T = len(off) // 2
    sel = [pix[off[0]:off[T]], pix[off[T]:off[2 * T]]]
    for v in range(2):
        xs, ys = sel[v] % 40, sel[v] // 40
        rgb, tf, fl = oracle.render_pixels(sc, cams, v, xs, ys)
        ok = fl == 0
        assert np.allclose(rgb[ok], full["images"][v][:, ys, xs].T[ok], rtol=1e-12, atol=1e-12)
    # dL/dimage split into the selection and the rest: gradients add up
    rng = np.random.default_rng(5)
    dl = [rng.normal(size=(3, 24, 40)) for _ in cams]
    part = [np.zeros_like(d) for d in dl]
    rest = [d.copy() for d in dl]
    for v in range(2):
        ys, xs = sel[v] // 40, sel[v] % 40
        part[v][:, ys, xs] = dl[v][:, ys, xs]
        rest[v][:, ys, xs] = 0.0
    a = oracle.backward(sc, cams, part, (8, 8))
    b = oracle.backward(sc, cams, rest, (8, 8))
    c = oracle.backward(sc, cams, dl, (8, 8))
    for n in ("means", "scales", "quats", "opacities", "sh"):
        assert np.allclose(a[n] + b[n], c[n], rtol=1e-9, atol=1e-12 * np.abs(c[n]).max())
