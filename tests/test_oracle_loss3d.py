"""The oracle's blended depth and 3D distance-aware D-SSIM (Sec. 5.1.2), pinned by closed forms,
a reduction to the 2D SSIM, an explicit per-pixel evaluation and finite differences."""
import numpy as np

import oracle
from paper_2506_12727_amd import scenes


def _one_gaussian_scene(pos, scale=0.08, opacity=0.7, n=1):
    sc = scenes.make_scene(n, 0)
    sc.means[:] = np.asarray(pos, np.float32)
    sc.scales[:] = scale
    sc.quats[:] = np.array([1, 0, 0, 0], np.float32)
    sc.opacities[:] = opacity
    sc.sh[:] = 0.3
    return sc


def test_depth_of_one_gaussian_is_its_depth():
    sc = _one_gaussian_scene([0.05, -0.02, 0.1])
    cams = [scenes.make_camera(48, 40, (0.0, 0.0, -3.0))]
    f = oracle.forward(sc, cams, (16, 16))
    z = float(oracle.geom32(sc, cams, 0)["depth"][0])
    a = 1.0 - f["t_final"][0]
    m = a > 1e-3
    assert m.sum() > 20
    assert np.allclose(f["depth"][0][m] / a[m], z, rtol=1e-12)
    assert np.all(f["depth"][0][~(a > 0)] == 0.0)


def test_depth_of_two_gaussians_composites_front_to_back():
    front = _one_gaussian_scene([0.0, 0.0, -0.3])
    back = _one_gaussian_scene([0.03, 0.0, 0.4], scale=0.12, opacity=0.6)
    both = scenes.make_scene(2, 0)
    for k, s in enumerate((front, back)):
        for n in ("means", "scales", "quats", "opacities", "sh"):
            getattr(both, n)[k] = getattr(s, n)[0]
    cams = [scenes.make_camera(40, 40, (0.0, 0.0, -3.0))]
    fa, fb, f2 = (oracle.forward(s, cams, (8, 8)) for s in (front, back, both))
    z = oracle.geom32(both, cams, 0)["depth"]
    a1, a2 = 1.0 - fa["t_final"][0], 1.0 - fb["t_final"][0]
    want = z[0] * a1 + z[1] * a2 * (1.0 - a1)
    assert np.allclose(f2["depth"][0], want, rtol=1e-12, atol=1e-15)


def test_depth_of_a_plane_facing_the_camera():
    sc = scenes.make_scene(300, 0, log_scale_mean=-2.8)
    sc.means[:, 2] = 0.0           # every mean on the plane z = 0, seen from (0, 0, -3)
    cams = [scenes.make_camera(64, 48, (0.0, 0.0, -3.0))]
    f = oracle.forward(sc, cams, (16, 16))
    z = oracle.geom32(sc, cams, 0)["depth"].astype(np.float64)
    p = oracle.geom32(sc, cams, 0)["participates"] == 1
    a = 1.0 - f["t_final"][0]
    m = a > 1e-3
    zbar = f["depth"][0][m] / a[m]
    assert zbar.min() >= z[p].min() - 1e-9 and zbar.max() <= z[p].max() + 1e-9
    assert abs(zbar.mean() - 3.0) < 1e-5


def test_surface_points_project_back_to_their_pixels():
    cams = scenes.make_cameras([(20, 14), (20, 14)], seed=4)
    rng = np.random.default_rng(2)
    vm = rng.integers(0, 2, size=(14, 20))
    tf = rng.uniform(0.0, 0.9, size=(14, 20))
    tf[3, 4] = 1.0                      # nothing blended: no point
    zbar = rng.uniform(1.0, 5.0, size=(14, 20))
    depth = zbar * (1.0 - tf)
    P, S = oracle.surface_points(cams, vm, depth, tf)
    assert S[3, 4] == 0.0 and np.all(P[3, 4] == 0.0)
    for y in range(14):
        for x in range(20):
            if (y, x) == (3, 4):
                continue
            c = cams[vm[y, x]]
            R = np.asarray(c.R, np.float64).reshape(3, 3)
            pc = R @ P[y, x] + np.asarray(c.t, np.float64)
            # (the float32 rotation is orthonormal to ~1e-7 only)
            assert abs(pc[2] - zbar[y, x]) < 1e-6 * zbar[y, x]
            assert abs(c.fx * pc[0] / pc[2] + c.cx - (x + 0.5)) < 1e-4
            assert abs(c.fy * pc[1] / pc[2] + c.cy - (y + 0.5)) < 1e-4
            assert abs(S[y, x] - 1.5 * zbar[y, x] / c.fx) < 1e-12


def _plane(W, H, z0=2.5):
    cams = [scenes.make_camera(W, H, (0.0, 0.0, -2.0))]
    tf = np.full((H, W), 0.25)
    return cams, np.zeros((H, W), int), z0 * (1.0 - tf), tf


def test_fronto_parallel_single_view_is_the_2d_ssim():
    W, H = 30, 24
    cams, vm, depth, tf = _plane(W, H)
    P, S = oracle.surface_points(cams, vm, depth, tf)
    rng = np.random.default_rng(6)
    a, b = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    _, _, s3 = oracle.loss3d(a, b, P, S, 0.0, 1.0)
    s2 = np.stack([oracle.ssim_map(a[ch], b[ch]) for ch in range(3)])
    r = oracle.SSIM3D_RADIUS
    assert np.allclose(s3[:, r:H - r, r:W - r], s2[:, r:H - r, r:W - r], rtol=1e-9, atol=1e-12)


def test_identical_images_have_no_dssim():
    W, H = 16, 12
    cams = scenes.make_cameras([(W, H), (W, H)], seed=3)
    rng = np.random.default_rng(1)
    vm = rng.integers(0, 2, size=(H, W))
    tf = rng.uniform(0.0, 0.5, size=(H, W))
    depth = rng.uniform(1.0, 4.0, size=(H, W)) * (1.0 - tf)
    P, S = oracle.surface_points(cams, vm, depth, tf)
    a = rng.uniform(size=(3, H, W))
    loss, grad, s = oracle.loss3d(a, a, P, S, 0.0, 1.0)
    assert abs(loss) < 1e-12 and np.abs(grad).max() < 1e-12 and np.allclose(s, 1.0)


def _explicit_ssim3d(a, b, P, S, y, x, ch):
    """SSIM* at one centre by a direct loop over its window."""
    H, W = S.shape
    r = oracle.SSIM3D_RADIUS
    sw = s1 = s2 = s11 = s22 = s12 = 0.0
    for qy in range(y - r, y + r + 1):
        for qx in range(x - r, x + r + 1):
            if not (0 <= qy < H and 0 <= qx < W):
                continue
            if S[y, x] > 0:
                if not S[qy, qx] > 0:
                    continue
                d2 = float(((P[qy, qx] - P[y, x]) ** 2).sum())
                w = np.exp(-d2 / (2.0 * S[y, x] ** 2))
            else:
                w = 1.0 if (qy, qx) == (y, x) else 0.0
            u, v = a[ch, qy, qx], b[ch, qy, qx]
            sw += w; s1 += w * u; s2 += w * v; s11 += w * u * u; s22 += w * v * v; s12 += w * u * v
    m1, m2 = s1 / sw, s2 / sw
    v1, v2, c12 = s11 / sw - m1 * m1, s22 / sw - m2 * m2, s12 / sw - m1 * m2
    C1, C2 = oracle.SSIM_C1, oracle.SSIM_C2
    return (2 * m1 * m2 + C1) * (2 * c12 + C2) / ((m1 * m1 + m2 * m2 + C1) * (v1 + v2 + C2))


def test_matches_an_explicit_loop_on_a_mixed_plane():
    W, H = 13, 10
    cams = scenes.make_cameras([(W, H), (W, H), (W, H)], seed=8)
    rng = np.random.default_rng(9)
    vm = rng.integers(0, 3, size=(H, W))
    tf = rng.uniform(0.0, 0.6, size=(H, W))
    tf[rng.uniform(size=(H, W)) < 0.08] = 1.0     # some pixels without a surface
    depth = rng.uniform(1.5, 3.0, size=(H, W)) * (1.0 - tf)
    P, S = oracle.surface_points(cams, vm, depth, tf)
    a, b = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    _, _, s = oracle.loss3d(a, b, P, S, 0.0, 1.0)
    for y in range(H):
        for x in range(W):
            for ch in range(3):
                assert abs(s[ch, y, x] - _explicit_ssim3d(a, b, P, S, y, x, ch)) < 1e-10


def test_far_apart_views_do_not_mix():
    """Two views on a checkerboard, one surface near and one far: every window only averages the
    pixels of its own view, as if the other view's pixels were not in the plane."""
    W, H = 14, 12
    cams = [scenes.make_camera(W, H, (0.0, 0.0, -2.0)), scenes.make_camera(W, H, (0.0, 0.0, -2.0))]
    vm = (np.add.outer(np.arange(H), np.arange(W)) % 2)
    tf = np.full((H, W), 0.3)
    depth = np.where(vm == 0, 1.0, 400.0) * (1.0 - tf)
    P, S = oracle.surface_points(cams, vm, depth, tf)
    rng = np.random.default_rng(4)
    a, b = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    _, _, s = oracle.loss3d(a, b, P, S, 0.0, 1.0)
    # the same plane with the other view's pixels removed (no point, so they never enter a window)
    for v in (0, 1):
        S_only = np.where(vm == v, S, 0.0)
        for y in range(H):
            for x in range(W):
                if vm[y, x] != v:
                    continue
                assert abs(s[0, y, x] - _explicit_ssim3d(a, b, P, S_only, y, x, 0)) < 1e-9


def test_gradient_by_finite_differences():
    W, H = 12, 9
    cams = scenes.make_cameras([(W, H), (W, H)], seed=5)
    rng = np.random.default_rng(10)
    vm = rng.integers(0, 2, size=(H, W))
    tf = rng.uniform(0.0, 0.6, size=(H, W))
    depth = rng.uniform(1.5, 3.0, size=(H, W)) * (1.0 - tf)
    P, S = oracle.surface_points(cams, vm, depth, tf)
    a, b = rng.uniform(size=(3, H, W)), rng.uniform(size=(3, H, W))
    for wl1, wd in [(0.8, 0.2), (0.0, 1.0)]:
        _, g, _ = oracle.loss3d(a, b, P, S, wl1, wd)
        h = 1e-6
        for _ in range(25):
            idx = (int(rng.integers(3)), int(rng.integers(H)), int(rng.integers(W)))
            if abs(a[idx] - b[idx]) < 1e-3:
                continue   # the L1 kink
            ap, am = a.copy(), a.copy()
            ap[idx] += h
            am[idx] -= h
            fd = (oracle.loss3d(ap, b, P, S, wl1, wd)[0] - oracle.loss3d(am, b, P, S, wl1, wd)[0]) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * abs(fd) + 1e-10, (idx, fd, g[idx])
