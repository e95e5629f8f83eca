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
                ("cut", C.c_float), ("hi", C.c_float),
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
        L.ora_forward.argtypes = [vp, vp, i32, i32, d, vp, vp, vp, vp, vp, vp]
        L.ora_backward.argtypes = [vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.ora_project64.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.ora_render_pixels.argtypes = [vp, vp, i32, i32, d, i64, vp, vp, vp, vp, vp, vp]
        L.ora_count_pairs.argtypes = [vp, vp, vp, vp]
        L.ora_loss.argtypes = [vp, vp, vp, d, d, vp, vp]
        L.ora_ssim_map.argtypes = [i32, i32, vp, vp, vp]
        L.ora_sh_basis.argtypes = [C.c_int, vp, vp, vp]
        L.ora_sh_count.restype = C.c_int
        L.ora_set_threads.argtypes = [i32]
        L.ora_set_threads.restype = None
        L.ora_max_threads.restype = i32
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


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().ora_set_threads(int(n))


def max_threads() -> int:
    return int(lib().ora_max_threads())


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


# Relative margin of the transmittance stop test (T' against 1e-4) within which a pixel is flagged:
# the kernel's single-precision transmittance was measured within 2e-6 relative of the oracle's on
# the parity scenes; 2e-5 keeps ten times that.
STOP_MARGIN = 2e-5


def forward(scene, cams, tile=(16, 16), geom32_mode=True, brute_force=False, margin=STOP_MARGIN):
    """Images [3,H,W] (float64), T_final [H,W], blended depth [H,W] (sum of z alpha T over the
    blended Gaussians, z camera-space depth), contributor counts, per-pixel flags and a per-view
    hash of every discrete decision taken.

    Every per-pixel decision (the cut test power >= max(-4.5, -ln(255 o)), the clamp power >
    ln(0.99 / o), the stop T' < 1e-4) is taken in double precision. geom32_mode=True blends with
    the single-precision projected mean and conic (the geometry the kernel blends with: image
    parity at 1e-5 needs it); False with the double projection (gradient parity). Flags: bit 0 the
    stop test is within `margin` relative of its threshold, bit 1 a cut or clamp test is within
    the single-precision error of the power (in double mode also plus the power's change between
    the double and the single-precision geometry). Flagged pixels may be decided otherwise by the
    kernel and are excluded from comparisons."""
    s, c = OScene(scene), OCams(cams, tile)
    imgs = [np.zeros((3, h, w)) for (w, h) in c.sizes]
    tf = [np.zeros((h, w)) for (w, h) in c.sizes]
    dp = [np.zeros((h, w)) for (w, h) in c.sizes]
    nc = [np.zeros((h, w), np.int32) for (w, h) in c.sizes]
    fl = [np.zeros((h, w), np.uint8) for (w, h) in c.sizes]
    th = np.zeros(c.B, np.uint64)
    ss, cs = s.struct(), c.struct()
    lib().ora_forward(C.byref(ss), C.byref(cs), int(geom32_mode), int(brute_force), float(margin),
                      _ptrs(imgs), _ptrs(tf), _ptrs(dp), _ptrs(nc), _ptrs(fl), _ptr(th))
    return dict(images=imgs, t_final=tf, depth=dp, n_contrib=nc, flags=fl, trace=th)


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


def backward(scene, cams, dl_dimg, tile=(16, 16), geom32_mode=False, want_mean2d=False):
    """Gradients of the loss whose image gradients are `dl_dimg` (list of [3,H,W]) with respect to
    means, scales, quats, opacities and SH, plus the densification statistics E1, E2, count and
    the comparator E_old. Double-precision geometry by default (geom32_mode=False); the per-pixel
    decisions as in forward(); pixels flagged by forward(..., geom32_mode) should carry zero image
    gradient on both sides of a comparison."""
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


def render_pixels(scene, cams, v: int, xs, ys, geom32_mode=True, margin=STOP_MARGIN, with_depth=False):
    """Colour [n,3], final transmittance [n] and flags [n] (and, with_depth, the blended depth [n]
    after them) of chosen pixels of view v, each by a walk over every participating Gaussian in
    depth order (usable at any scene size)."""
    s, c = OScene(scene), OCams(cams)
    xs = np.ascontiguousarray(xs, np.int32); ys = np.ascontiguousarray(ys, np.int32)
    n = len(xs)
    rgb = np.zeros((n, 3)); tf = np.zeros(n); dp = np.zeros(n); fl = np.zeros(n, np.uint8)
    ss, cs = s.struct(), c.struct()
    lib().ora_render_pixels(C.byref(ss), C.byref(cs), v, int(geom32_mode), float(margin), n, _ptr(xs), _ptr(ys),
                            _ptr(rgb), _ptr(tf), _ptr(dp), _ptr(fl))
    if with_depth:
        return rgb, tf, fl, dp
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
    [offsets[s], offsets[s+1]) of `pixels` lists, in ascending position, the pixel indices
    y*width + x of view v in tile t, with s = v * tiles_per_view + t (tiles row-major within a
    view). (The order inside a segment does not change what is rendered.) Plain loops, one tile at
    a time."""
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
            for v in range(B):
                segs[v * T + t].sort()
    offsets = np.zeros(B * T + 1, np.uint32)
    offsets[1:] = np.cumsum([len(s) for s in segs])
    pixels = np.array([p for s in segs for p in s], dtype=np.uint32)
    return offsets, pixels


# ---------------------------------------------------------------------------------------------
# 3D distance-aware D-SSIM (Sec. 5.1.2, Eqs. 7-11), on the merged image plane of partial rendering
# ---------------------------------------------------------------------------------------------

SSIM3D_SIGMA_PX = 1.5     # the window's sigma in pixels, as in the 2D D-SSIM
SSIM3D_RADIUS = 5         # 11 x 11 window
SSIM_C1, SSIM_C2 = 0.01 ** 2, 0.03 ** 2


def surface_points(cams, view_map, depth, t_final):
    """World-space surface point of every pixel of a merged image plane.

    Pixel (x, y) was rendered from view view_map[y, x]. Its surface depth is the blended depth over
    the blended opacity, zbar = depth / (1 - T_final), defined where something was blended
    (T_final < 1); the point is R^T (zbar * ((x + 0.5 - cx) / fx, (y + 0.5 - cy) / fy, 1) - t), the
    pixel-to-world map of the 3D kernel's definition. Also returns the kernel's width at the point:
    1.5 pixels at depth zbar in world units, 1.5 zbar / fx (0 where there is no point).
    Returns (points [H, W, 3], scale [H, W])."""
    view_map = np.asarray(view_map)
    H, W = view_map.shape
    P = np.zeros((H, W, 3))
    S = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            c = cams[int(view_map[y, x])]
            a = 1.0 - float(t_final[y, x])
            if not a > 0.0:
                continue
            z = float(depth[y, x]) / a
            ray = np.array([(x + 0.5 - c.cx) / c.fx, (y + 0.5 - c.cy) / c.fy, 1.0])
            R = np.asarray(c.R, np.float64).reshape(3, 3)
            t = np.asarray(c.t, np.float64).reshape(3)
            P[y, x] = R.T @ (z * ray - t)
            S[y, x] = SSIM3D_SIGMA_PX * z / c.fx
    return P, S


def _kernel3d(points, scale, du, dv):
    """Weights w[c] of the window offset (du, dv) for every centre c: exp(-|P(c + d) - P(c)|^2 /
    (2 scale(c)^2)) where both pixels have points and c + d is inside the plane; a centre without a
    point keeps only itself. Returns (w [H, W], q index arrays (qy, qx) clipped, inside mask)."""
    H, W = scale.shape
    ys, xs = np.mgrid[0:H, 0:W]
    qy, qx = ys + dv, xs + du
    inside = (qy >= 0) & (qy < H) & (qx >= 0) & (qx < W)
    qyc, qxc = np.clip(qy, 0, H - 1), np.clip(qx, 0, W - 1)
    has_c = scale > 0
    has_q = scale[qyc, qxc] > 0
    d2 = ((points[qyc, qxc] - points) ** 2).sum(-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        w = np.where(has_c & has_q, np.exp(-d2 / (2.0 * np.where(has_c, scale, 1.0) ** 2)), 0.0)
    if du == 0 and dv == 0:
        w = np.where(has_c, w, 1.0)
    return np.where(inside, w, 0.0), qyc, qxc


def loss3d(image, target, points, scale, w_l1=1.0, w_dssim=0.0):
    """L = w_l1 mean|I - T| + w_dssim (1 - mean SSIM*) over one merged plane [3, H, W], where
    SSIM* is Eqs. 7-10 with the window replaced by the 3D distance-aware kernel (Eq. 11) around each
    centre, normalised to sum 1 over the in-plane window. The kernel's weights are constants (the
    rendered depth passes no gradient). Returns (loss, dL/dimage [3, H, W])."""
    I1 = np.asarray(image, np.float64)
    I2 = np.asarray(target, np.float64)
    _, H, W = I1.shape
    N = I1.size
    r = SSIM3D_RADIUS
    offs = [(du, dv) for dv in range(-r, r + 1) for du in range(-r, r + 1)]
    Wc = np.zeros((H, W))
    m1 = np.zeros_like(I1); m2 = np.zeros_like(I1)
    e11 = np.zeros_like(I1); e22 = np.zeros_like(I1); e12 = np.zeros_like(I1)
    for du, dv in offs:
        w, qy, qx = _kernel3d(points, scale, du, dv)
        a, b = I1[:, qy, qx], I2[:, qy, qx]
        Wc += w
        m1 += w * a; m2 += w * b
        e11 += w * a * a; e22 += w * b * b; e12 += w * a * b
    mu1, mu2 = m1 / Wc, m2 / Wc
    s11 = e11 / Wc - mu1 * mu1
    s22 = e22 / Wc - mu2 * mu2
    s12 = e12 / Wc - mu1 * mu2
    A = 2 * mu1 * mu2 + SSIM_C1
    Bn = 2 * s12 + SSIM_C2
    Cn = mu1 * mu1 + mu2 * mu2 + SSIM_C1
    Dn = s11 + s22 + SSIM_C2
    S = A * Bn / (Cn * Dn)
    L1 = np.abs(I1 - I2).mean()
    loss = w_l1 * L1 + w_dssim * (1.0 - S.mean())
    # dS(c)/dI1(q) = w_cq / W_c * (dS/dmu1 + dS/ds11 * 2 (I1(q) - mu1) + dS/ds12 * (I2(q) - mu2))
    dmu = 2 * mu2 * Bn / (Cn * Dn) - S * 2 * mu1 / Cn
    ds11 = -S / Dn
    ds12 = 2 * A / (Cn * Dn)
    ca = (dmu - 2 * mu1 * ds11 - mu2 * ds12) / Wc
    cb = 2 * ds11 / Wc
    cd = ds12 / Wc
    dS = np.zeros_like(I1)
    ys, xs = np.mgrid[0:H, 0:W]
    for du, dv in offs:
        w, qy, qx = _kernel3d(points, scale, du, dv)
        contrib = w * (ca + cb * I1[:, qy, qx] + cd * I2[:, qy, qx])
        inside = w > 0
        np.add.at(dS, (slice(None), qy[inside], qx[inside]), contrib[:, inside])
    grad = w_l1 * np.sign(I1 - I2) / N - w_dssim * dS / N
    return loss, grad, S


# ---------------------------------------------------------------------------------------------
# Multi-view adaptive density control (Sec. 5.2.2 with the statistics of Eqs. 13-14)
# ---------------------------------------------------------------------------------------------

def densify(means, scales, quats, opacities, sh, e1, e2, count, normals, split_threshold, clone_threshold,
            dense_scale, min_opacity):
    """One densification step over activated parameters. Per Gaussian g with count[g] > 0:
    mean E1 = e1/count above split_threshold and largest scale above dense_scale -> split into two
    children drawn from the Gaussian itself (means mu + R (s * z_k) with z_k = normals[g, k], the
    normalised quaternion's rotation R, scales s / 1.6, other parameters copied); mean E2 =
    e2/count above clone_threshold and largest scale at most dense_scale -> clone (the original
    and an identical copy). A Gaussian with opacity below min_opacity is pruned with all it would
    produce. Outputs keep the order of the originals (each original's outputs in a row: itself,
    its copy, or its two children). The decisions are compared in single precision; the children's
    means in double. Returns (means, scales, quats, opacities, sh, src) with src the original index
    of each output."""
    P = len(means)
    out = {k: [] for k in ("means", "scales", "quats", "opacities", "sh", "src")}

    def emit(g, mu, s):
        out["means"].append(np.asarray(mu, np.float64))
        out["scales"].append(np.asarray(s, np.float64))
        out["quats"].append(np.asarray(quats[g], np.float64))
        out["opacities"].append(float(opacities[g]))
        out["sh"].append(np.asarray(sh[g], np.float64))
        out["src"].append(g)

    f32 = np.float32
    for g in range(P):
        # the decisions are taken in single precision, as the kernels take them
        if f32(opacities[g]) < f32(min_opacity):
            continue
        s = np.asarray(scales[g], np.float64)
        big = f32(np.max(np.asarray(scales[g], f32))) > f32(dense_scale)
        c = int(count[g])
        m1 = f32(f32(e1[g]) / f32(c)) if c > 0 else f32(0.0)
        m2 = f32(f32(e2[g]) / f32(c)) if c > 0 else f32(0.0)
        if big and m1 > f32(split_threshold):
            w, x, y, z = np.asarray(quats[g], np.float64) / np.linalg.norm(np.asarray(quats[g], np.float64))
            R = np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                          [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                          [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])
            for k in range(2):
                emit(g, np.asarray(means[g], np.float64) + R @ (s * np.asarray(normals[g][k], np.float64)), s / 1.6)
        elif (not big) and m2 > f32(clone_threshold):
            emit(g, means[g], s)
            emit(g, means[g], s)
        else:
            emit(g, means[g], s)
    res = [np.array(out[k]) for k in ("means", "scales", "quats")]
    res.append(np.array(out["opacities"]))
    res.append(np.array(out["sh"]).reshape((-1,) + np.asarray(sh).shape[1:]))
    res.append(np.array(out["src"], np.int64))
    return tuple(res)


def adam_step(params, grads, moments, step, lr, beta1=0.9, beta2=0.999, eps=1e-15):
    """One Adam step (Kingma and Ba; the optimiser 3DGS trains with) of activated parameters, in
    double precision, returning new (params, moments). params and grads: dicts of means [P,3],
    scales [P,3], quats [P,4], opacities [P], sh [P,K,3] (grads with respect to the activated
    values). Scales and opacities move in log-scale and logit coordinates: their gradients pass
    through exp and the sigmoid, the step is applied there and mapped back (opacities of exactly
    0 or 1 stay). moments: [P, 11 + 3K, 2] (m, v), per Gaussian in the order means, scales,
    quats, opacity, SH. lr: dict(means, scales, quats, opacities, sh_dc, sh_rest)."""
    P = len(params["means"])
    K = np.asarray(params["sh"]).shape[1]
    d = lambda a: np.asarray(a, np.float64)
    s, o = d(params["scales"]), d(params["opacities"]).reshape(P)
    # gradient in the optimised coordinates, per Gaussian in the moment order
    gvec = np.concatenate([d(grads["means"]).reshape(P, 3), (d(grads["scales"]) * s).reshape(P, 3),
                           d(grads["quats"]).reshape(P, 4), (d(grads["opacities"]).reshape(P) * o * (1 - o))[:, None],
                           d(grads["sh"]).reshape(P, 3 * K)], axis=1)
    lrs = np.concatenate([np.full(3, lr["means"]), np.full(3, lr["scales"]), np.full(4, lr["quats"]),
                          [lr["opacities"]], np.full(3, lr["sh_dc"]), np.full(3 * K - 3, lr["sh_rest"])])
    mom = d(moments).copy()
    m = beta1 * mom[..., 0] + (1 - beta1) * gvec
    v = beta2 * mom[..., 1] + (1 - beta2) * gvec * gvec
    mom[..., 0], mom[..., 1] = m, v
    stepv = lrs[None, :] * (m / (1 - beta1 ** step)) / (np.sqrt(v / (1 - beta2 ** step)) + eps)
    out = dict(means=d(params["means"]) - stepv[:, 0:3], scales=s * np.exp(-stepv[:, 3:6]),
               quats=d(params["quats"]) - stepv[:, 6:10], sh=(d(params["sh"]).reshape(P, 3 * K) - stepv[:, 11:])
               .reshape(P, K, 3))
    inner = (o > 0) & (o < 1)
    logit = np.log(np.where(inner, o, 0.5)) - np.log1p(-np.where(inner, o, 0.5))
    out["opacities"] = np.where(inner, 1.0 / (1.0 + np.exp(-(logit - stepv[:, 10]))), o)
    return out, mom


def flatten_grads(g) -> np.ndarray:
    """The gradient vector of Sec. 3.2's variance: means | scales | quats | opacities | SH."""
    return np.concatenate([np.asarray(g[k], np.float64).reshape(-1)
                           for k in ("means", "scales", "quats", "opacities", "sh")])


def minibatch_variance(vectors) -> float:
    """Monte Carlo estimate of the variance of mini-batch gradients (Sec. 3.2): the mean squared
    norm of the sampled mini-batch gradients minus the squared norm of their mean."""
    x = np.asarray(vectors, np.float64)
    return float(np.mean(np.sum(x * x, axis=1)) - np.sum(np.mean(x, axis=0) ** 2))


def batch_gradient(scene, cams, targets, views, w_l1=1.0, tile=(16, 16)):
    """Gradient of the mini-batch loss formed by the listed views: the mean over those views of
    each view's mean L1 loss (the loss whose expectation over uniformly drawn views is the loss
    over the whole set)."""
    sub = [cams[v] for v in views]
    imgs = forward(scene, sub, tile)["images"]
    dl = []
    for img, v in zip(imgs, views):
        t = np.asarray(targets[v], np.float64)
        n = t.size
        dl.append(w_l1 * np.sign(img - t) / (n * len(views)))
    return backward(scene, sub, dl, tile)


def partial_batch_gradient(scene, cams, targets, views, keys, tile=(16, 16)):
    """Gradient of the L1 loss of one partial-rendering mini-batch (Alg. 3): the listed views (of
    one size) share the image plane by the sub-sampling of `keys`; each pixel of the plane is
    rendered from the view that took it and compared with that view's target; the loss is the
    mean over the plane's (channel, row, column)."""
    sub = [cams[v] for v in views]
    W, H = sub[0].width, sub[0].height
    off, pix = subsample_tiles(W, H, len(views), tile, keys)
    T = (len(off) - 1) // len(views)
    imgs = forward(scene, sub, tile)["images"]
    dl = []
    for j, v in enumerate(views):
        sel = pix[off[j * T]:off[(j + 1) * T]]
        ys, xs = sel // W, sel % W
        d = np.zeros((3, H, W))
        diff = imgs[j][:, ys, xs] - np.asarray(targets[v], np.float64)[:, ys, xs]
        d[:, ys, xs] = np.sign(diff) / (3 * W * H)
        dl.append(d)
    return backward(scene, sub, dl, tile)
