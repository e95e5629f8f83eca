"""Python access to the CPU oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE ONLY. The oracle is the plain double-precision reference
rasterizer that the GPU path is checked against; only the tests, the smoke check
and the CPU-baseline leg of the benchmark may import it. It imports nothing from
the GPU package: scenes and cameras are taken by duck typing (objects with
means/scales/quats/opacities/sh/sh_degree, and width/height/fx/fy/cx/cy/R/t/bg).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class _Cams(C.Structure):
    _fields_ = [("B", C.c_int32), ("tile_w", C.c_int32), ("tile_h", C.c_int32),
                ("wh", C.c_void_p), ("intr", C.c_void_p), ("R", C.c_void_p), ("t", C.c_void_p),
                ("bg", C.c_void_p)]


class _Scene(C.Structure):
    _fields_ = [("P", C.c_int64), ("sh_degree", C.c_int32), ("means", C.c_void_p), ("scales", C.c_void_p),
                ("quats", C.c_void_p), ("opac", C.c_void_p), ("sh", C.c_void_p)]


class G32(C.Structure):
    _fields_ = [("participates", C.c_int32), ("depth", C.c_float), ("depth_bits", C.c_uint32),
                ("mx", C.c_float), ("my", C.c_float), ("ca", C.c_float), ("cb", C.c_float), ("cc", C.c_float),
                ("hca", C.c_float), ("nb", C.c_float), ("hcc", C.c_float), ("cut", C.c_float), ("hi", C.c_float),
                ("radius", C.c_float), ("x0", C.c_int32), ("x1", C.c_int32), ("y0", C.c_int32), ("y1", C.c_int32)]


G32_DTYPE = np.dtype([(n, np.int32 if t in (C.c_int32,) else (np.uint32 if t is C.c_uint32 else np.float32))
                      for n, t in G32._fields_])


def lib():
    """Load liboracle.so, building it first only if it is not there."""
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.ora_ln32.restype = C.c_float
        L.ora_ln32.argtypes = [C.c_float]
        L.ora_geom32_view.argtypes = [vp, vp, i32, vp]
        L.ora_total_tiles.restype = i64
        L.ora_total_tiles.argtypes = [vp]
        L.ora_binning.restype = i64
        L.ora_binning.argtypes = [vp, vp, vp, vp, i64, vp]
        L.ora_forward.argtypes = [vp, vp, i32, i32, d, vp, vp, vp, vp, vp]
        L.ora_backward.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ora_project64.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.ora_render_pixels.argtypes = [vp, vp, i32, i32, d, i64, vp, vp, vp, vp, vp]
        L.ora_count_pairs.argtypes = [vp, vp, vp, vp]
        L.ora_loss.argtypes = [vp, vp, vp, d, d, vp, vp]
        L.ora_ssim_map.argtypes = [i32, i32, vp, vp, vp]
        L.ora_sh_basis.argtypes = [C.c_int, vp, vp, vp]
        L.ora_sh_count.restype = C.c_int
        _LIB = L
    return _LIB


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _ptrs(arrs: Sequence[np.ndarray]):
    out = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    return out


class OScene:
    """Double-precision copy of a scene (keeps the arrays alive for the C struct)."""

    def __init__(self, scene):
        f = lambda a: np.ascontiguousarray(np.asarray(a, np.float64))
        self.means, self.scales, self.quats = f(scene.means), f(scene.scales), f(scene.quats)
        self.opac = f(scene.opacities).reshape(-1)
        self.sh_degree = int(scene.sh_degree)
        self.sh = f(scene.sh).reshape(self.means.shape[0], -1, 3)
        self.P = self.means.shape[0]

    def struct(self) -> _Scene:
        return _Scene(self.P, self.sh_degree, _ptr(self.means), _ptr(self.scales), _ptr(self.quats),
                      _ptr(self.opac), _ptr(self.sh))


class OCams:
    def __init__(self, cams, tile=(16, 16)):
        self.B = len(cams)
        self.wh = np.ascontiguousarray([[c.width, c.height] for c in cams], np.int32).reshape(-1)
        self.intr = np.ascontiguousarray([[c.fx, c.fy, c.cx, c.cy] for c in cams], np.float64).reshape(-1)
        self.R = np.ascontiguousarray([np.asarray(c.R, np.float64).reshape(9) for c in cams]).reshape(-1)
        self.t = np.ascontiguousarray([np.asarray(c.t, np.float64).reshape(3) for c in cams]).reshape(-1)
        self.bg = np.ascontiguousarray([np.asarray(c.bg, np.float64).reshape(3) for c in cams]).reshape(-1)
        self.tile = tile
        self.sizes = [(int(c.width), int(c.height)) for c in cams]

    def struct(self) -> _Cams:
        return _Cams(self.B, self.tile[0], self.tile[1], _ptr(self.wh), _ptr(self.intr), _ptr(self.R),
                     _ptr(self.t), _ptr(self.bg))

    def total_tiles(self) -> int:
        return sum(((w + self.tile[0] - 1) // self.tile[0]) * ((h + self.tile[1] - 1) // self.tile[1])
                   for (w, h) in self.sizes)


def ln32(x: float) -> float:
    return float(lib().ora_ln32(float(x)))


def geom32(scene, cams, v: int, tile=(16, 16)) -> np.ndarray:
    s, c = OScene(scene), OCams(cams, tile)
    out = np.zeros(s.P, G32_DTYPE)
    ss, cs = s.struct(), c.struct()
    lib().ora_geom32_view(C.byref(ss), C.byref(cs), v, _ptr(out))
    return out


def project64(scene, cams, v: int):
    s, c = OScene(scene), OCams(cams)
    m = np.zeros((s.P, 2)); cov = np.zeros((s.P, 3)); rgb = np.zeros((s.P, 3)); z = np.zeros(s.P)
    ss, cs = s.struct(), c.struct()
    lib().ora_project64(C.byref(ss), C.byref(cs), v, _ptr(m), _ptr(cov), _ptr(rgb), _ptr(z))
    return m, cov, rgb, z


def binning(scene, cams, tile=(16, 16)):
    """Sorted 64-bit keys (view<<48 | tile<<32 | depth bits), values (Gaussian index) and
    per-(view, tile) [start, end) ranges (global tile order, view-major; empty tiles [0,0))."""
    s, c = OScene(scene), OCams(cams, tile)
    ss, cs = s.struct(), c.struct()
    K = int(lib().ora_binning(C.byref(ss), C.byref(cs), None, None, 0, None))
    keys = np.zeros(max(K, 1), np.uint64)
    vals = np.zeros(max(K, 1), np.uint32)
    ranges = np.zeros((c.total_tiles(), 2), np.uint32)
    lib().ora_binning(C.byref(ss), C.byref(cs), _ptr(keys), _ptr(vals), K, _ptr(ranges))
    return keys[:K], vals[:K], ranges


def forward(scene, cams, tile=(16, 16), geom32_mode=True, brute_force=False, margin=1e-4):
    """Images [3,H,W] (float64), T_final [H,W], contributor counts, per-pixel flags
    (bit 0: the transmittance stop is within `margin` relative of its threshold) and a per-view
    hash of every discrete decision taken."""
    s, c = OScene(scene), OCams(cams, tile)
    imgs = [np.zeros((3, h, w)) for (w, h) in c.sizes]
    tf = [np.zeros((h, w)) for (w, h) in c.sizes]
    nc = [np.zeros((h, w), np.int32) for (w, h) in c.sizes]
    fl = [np.zeros((h, w), np.uint8) for (w, h) in c.sizes]
    th = np.zeros(c.B, np.uint64)
    ss, cs = s.struct(), c.struct()
    lib().ora_forward(C.byref(ss), C.byref(cs), int(geom32_mode), int(brute_force), float(margin),
                      _ptrs(imgs), _ptrs(tf), _ptrs(nc), _ptrs(fl), _ptr(th))
    return dict(images=imgs, t_final=tf, n_contrib=nc, flags=fl, trace=th)


def loss(cams, images, targets, w_l1=1.0, w_dssim=0.0):
    c = OCams(cams)
    im = [np.ascontiguousarray(np.asarray(a, np.float64)) for a in images]
    tg = [np.ascontiguousarray(np.asarray(a, np.float64)) for a in targets]
    grads = [np.zeros_like(a) for a in im]
    out = np.zeros(1)
    cs = c.struct()
    lib().ora_loss(C.byref(cs), _ptrs(im), _ptrs(tg), float(w_l1), float(w_dssim), _ptr(out), _ptrs(grads))
    return float(out[0]), grads


def ssim_map(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, np.float64); b = np.ascontiguousarray(b, np.float64)
    H, W = a.shape
    out = np.zeros((H, W))
    lib().ora_ssim_map(W, H, _ptr(a), _ptr(b), _ptr(out))
    return out


def backward(scene, cams, dl_dimg, tile=(16, 16), geom32_mode=True, want_mean2d=False):
    """Gradients of the loss whose image gradients are `dl_dimg` (list of [3,H,W]) with respect to
    means, scales, quats, opacities and SH, plus the densification statistics E1, E2, count and
    the comparator E_old."""
    s, c = OScene(scene), OCams(cams, tile)
    P, K = s.P, (s.sh_degree + 1) ** 2
    g = dict(means=np.zeros((P, 3)), scales=np.zeros((P, 3)), quats=np.zeros((P, 4)), opacities=np.zeros(P),
             sh=np.zeros((P, K, 3)), e1=np.zeros(P), e2=np.zeros(P), count=np.zeros(P, np.int32),
             e_old=np.zeros(P))
    m2 = np.zeros((c.B, P, 2)) if want_mean2d else None
    dl = [np.ascontiguousarray(np.asarray(a, np.float64)) for a in dl_dimg]
    ss, cs = s.struct(), c.struct()
    lib().ora_backward(C.byref(ss), C.byref(cs), int(geom32_mode), _ptrs(dl), _ptr(g["means"]), _ptr(g["scales"]),
                       _ptr(g["quats"]), _ptr(g["opacities"]), _ptr(g["sh"]), _ptr(g["e1"]), _ptr(g["e2"]),
                       _ptr(g["count"]), _ptr(m2) if m2 is not None else None, _ptr(g["e_old"]))
    if m2 is not None:
        g["mean2d"] = m2
    return g


def sh_basis(degree: int, d) -> tuple:
    d = np.ascontiguousarray(np.asarray(d, np.float64).reshape(3))
    K = (degree + 1) ** 2
    Y = np.zeros(K)
    dY = np.zeros((K, 3))
    lib().ora_sh_basis(degree, _ptr(d), _ptr(Y), _ptr(dY))
    return Y, dY


def render_pixels(scene, cams, v: int, xs, ys, geom32_mode=True, margin=1e-4):
    """Colour [n,3], final transmittance [n] and flags [n] of chosen pixels of view v, each by a walk
    over every participating Gaussian in depth order (usable at any scene size)."""
    s, c = OScene(scene), OCams(cams)
    xs = np.ascontiguousarray(xs, np.int32); ys = np.ascontiguousarray(ys, np.int32)
    n = len(xs)
    rgb = np.zeros((n, 3)); tf = np.zeros(n); fl = np.zeros(n, np.uint8)
    ss, cs = s.struct(), c.struct()
    lib().ora_render_pixels(C.byref(ss), C.byref(cs), v, int(geom32_mode), float(margin), n, _ptr(xs), _ptr(ys),
                            _ptr(rgb), _ptr(tf), _ptr(fl))
    return rgb, tf, fl


def count_pairs(scene, cams, tile=(16, 16)):
    """(participating records, (Gaussian, tile) pairs) over the whole batch, without sorting."""
    s, c = OScene(scene), OCams(cams, tile)
    r = np.zeros(1, np.int64); p = np.zeros(1, np.int64)
    ss, cs = s.struct(), c.struct()
    lib().ora_count_pairs(C.byref(ss), C.byref(cs), _ptr(r), _ptr(p))
    return int(r[0]), int(p[0])


def subsample_tiles(width: int, height: int, B: int, tile, keys):
    """Index array of thread-efficient partial rendering (Alg. 3; Sec. 5.1.1) for B views of one
    size: each tile's pixel positions are shared out among the B views so that the views together
    cover the image plane once and each renders about N/B pixels of every tile (N pixels per tile).

    The sub-sampling draws one random key per pixel position (`keys`, [height*width] or
    [height, width], passed in): a tile's positions are ranked by (key, position index) and the
    position of rank r goes to view r mod B. Returns (offsets, pixels): segment
    [offsets[s], offsets[s+1]) of `pixels` lists, in rank order, the pixel indices y*width + x of
    view v in tile t, with s = v * tiles_per_view + t (tiles row-major within a view).
    Plain loops, one tile at a time."""
    tw, th = int(tile[0]), int(tile[1])
    W, H = int(width), int(height)
    keys = np.asarray(keys, dtype=np.uint32).reshape(-1)
    assert keys.size == W * H
    txn, tyn = (W + tw - 1) // tw, (H + th - 1) // th
    T = txn * tyn
    segs = [[] for _ in range(B * T)]
    for ty in range(tyn):
        for tx in range(txn):
            t = ty * txn + tx
            pos = [y * W + x for y in range(ty * th, min(H, ty * th + th))
                   for x in range(tx * tw, min(W, tx * tw + tw))]
            ranked = sorted(pos, key=lambda p: (int(keys[p]), p))
            for r, p in enumerate(ranked):
                segs[(r % B) * T + t].append(p)
    offsets = np.zeros(B * T + 1, np.uint32)
    offsets[1:] = np.cumsum([len(s) for s in segs])
    pixels = np.array([p for s in segs for p in s], dtype=np.uint32)
    return offsets, pixels
