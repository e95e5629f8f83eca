"""Pins of the oracle's projection and single-precision decision geometry against
closed forms, an independent rotation library and finite differences.

Paper passages: Sec. 3 (Sigma = R S S^T R^T; EWA projection to mu', Sigma'),
Appendix "Rasterization in multi-view training" (culling, tile duplication)."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from paper_2506_12727_amd import scenes


def _one(mean, scale, quat, opac=0.5, sh_dc=(0.0, 0.0, 0.0)):
    Y00 = 0.5 / math.sqrt(math.pi)
    # float64 arrays: the oracle's double-precision path sees these values exactly
    return scenes.Scene(np.asarray([mean], np.float64), np.asarray([scale], np.float64),
                        np.asarray([quat], np.float64), np.asarray([opac], np.float64),
                        np.asarray([[[c / Y00 for c in sh_dc]]], np.float64), 0)


def _cam(W=64, H=48, pos=(0, 0, -3.0)):
    return scenes.make_camera(W, H, pos)


def test_ln32_matches_log(ora):
    xs = np.concatenate([np.logspace(-38, 38, 2001), np.linspace(0.5, 2.0, 1001), [1.0, 255.0, 1 / 255.0]])
    for x in xs.astype(np.float32):
        got = ora.ln32(float(x))
        assert abs(got - math.log(float(x))) <= 2e-6 + 2e-7 * abs(math.log(float(x))), x
    assert ora.ln32(0.0) == -math.inf
    assert ora.ln32(-1.0) == -math.inf
    assert ora.ln32(float("nan")) == -math.inf
    assert ora.ln32(math.inf) == math.inf
    assert ora.ln32(1e-45) < -100  # subnormal input


def test_on_axis_point_projects_to_principal_point(ora):
    sc = _one((0, 0, 0), (0.05, 0.05, 0.05), (1, 0, 0, 0))
    cam = _cam()
    m, cov, rgb, z = ora.project64(sc, [cam], 0)
    assert np.allclose(m[0], [cam.cx, cam.cy], atol=1e-9)
    assert abs(z[0] - 3.0) < 1e-6
    g = ora.geom32(sc, [cam], 0)[0]
    assert g["participates"] == 1
    assert abs(g["mx"] - cam.cx) < 1e-4 and abs(g["my"] - cam.cy) < 1e-4


def test_isotropic_on_axis_closed_form(ora):
    # Sigma' = ((f s / z)^2 + 0.3) I for an isotropic Gaussian on the optical axis, any rotation
    s, zc = 0.05, 3.0
    cam = _cam()
    q = np.array([0.3, -0.5, 0.7, 0.2]); q /= np.linalg.norm(q)
    sc = _one((0, 0, 0), (s, s, s), q)
    m, cov, rgb, z = ora.project64(sc, [cam], 0)
    expect = (cam.fx * s / zc) ** 2 + 0.3
    assert np.allclose(cov[0], [expect, 0.0, expect], rtol=1e-6, atol=1e-9)
    g = ora.geom32(sc, [cam], 0)[0]
    assert abs(g["ca"] - 1 / expect) < 1e-6 / expect and abs(g["cb"]) < 1e-6
    r = math.ceil(3 * math.sqrt(expect))
    assert g["radius"] == r
    assert (g["x0"], g["x1"]) == (max(0, math.floor(cam.cx - r)), min(cam.width - 1, math.floor(cam.cx + r)))


def test_projection_jacobian_and_covariance_vs_independent_rotation(ora):
    """EWA: Sigma' - 0.3 I = (d mu'/d mu) Sigma (d mu'/d mu)^T with d mu'/d mu taken by central
    differences of the oracle's own projected mean, and Sigma built with scipy's rotation."""
    rng = np.random.default_rng(5)
    cams = scenes.make_cameras([(640, 480)], radius=3.0)
    for _ in range(20):
        mu = rng.uniform(-0.7, 0.7, 3)
        s = np.exp(rng.normal(-3, 0.5, 3))
        q = rng.normal(size=4)
        sc = _one(mu, s, q)
        m, cov, _, _ = ora.project64(sc, cams, 0)
        Jw = np.zeros((2, 3))
        h = 1e-6
        for k in range(3):
            e = np.zeros(3); e[k] = h
            mp = ora.project64(_one(mu + e, s, q), cams, 0)[0][0]
            mm = ora.project64(_one(mu - e, s, q), cams, 0)[0][0]
            Jw[:, k] = (mp - mm) / (2 * h)
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        S = np.diag(s)
        Sig = Rq @ S @ S @ Rq.T
        C2 = Jw @ Sig @ Jw.T
        assert np.allclose([C2[0, 0] + 0.3, C2[0, 1], C2[1, 1] + 0.3], cov[0], rtol=1e-5, atol=1e-6)


def test_rotation_identity_and_determinant(ora):
    cam = _cam()
    s = np.array([0.01, 0.03, 0.07])
    sc = _one((0, 0, 0), s, (1, 0, 0, 0))
    _, cov, _, _ = ora.project64(sc, [cam], 0)
    # identity rotation, camera axes aligned with world: Sigma' diagonal = (f/z)^2 * (s_x^2, s_y^2) + 0.3
    f, z = cam.fx, 3.0
    assert np.allclose(cov[0], [(f / z) ** 2 * s[0] ** 2 + 0.3, 0.0, (f / z) ** 2 * s[1] ** 2 + 0.3], rtol=1e-9)


def test_geom32_tracks_double_projection(ora):
    sc = scenes.make_scene(3000, 0)
    cams = scenes.make_cameras([(1280, 720), (200, 150)])
    for v in range(2):
        g = ora.geom32(sc, cams, v)
        m, cov, _, z = ora.project64(sc, cams, v)
        p = g["participates"] == 1
        assert p.sum() > 100
        assert np.all(np.abs(g["mx"][p] - m[p, 0]) <= 1e-5 * (np.abs(m[p, 0]) + 10))
        assert np.all(np.abs(g["my"][p] - m[p, 1]) <= 1e-5 * (np.abs(m[p, 1]) + 10))
        det = cov[:, 0] * cov[:, 2] - cov[:, 1] ** 2
        conic = np.stack([cov[:, 2] / det, -cov[:, 1] / det, cov[:, 0] / det], 1)
        for k, n in enumerate(["ca", "cb", "cc"]):
            assert np.allclose(g[n][p], conic[p, k], rtol=1e-4, atol=1e-5 * np.abs(conic[p]).max())
        assert np.all(g["depth"][p] > 0.2)
        bits = g["depth"].view(np.uint32)
        assert np.array_equal(bits, g["depth_bits"])


def test_participation_rules(ora):
    cam = _cam(64, 48, pos=(0, 0, -3.0))
    behind = _one((0, 0, -3.5), (0.05,) * 3, (1, 0, 0, 0))           # behind the camera
    near = _one((0, 0, -2.85), (0.05,) * 3, (1, 0, 0, 0))            # z = 0.15 < 0.2
    off = _one((3.0, 0, 0), (0.01,) * 3, (1, 0, 0, 0))              # far outside the image
    inside = _one((0.2, 0.1, 0), (0.01,) * 3, (1, 0, 0, 0))
    zeroq = _one((0, 0, 0), (0.05,) * 3, (0, 0, 0, 0))              # degenerate quaternion
    for sc, want in [(behind, 0), (near, 0), (off, 0), (inside, 1), (zeroq, 0)]:
        assert ora.geom32(sc, [cam], 0)[0]["participates"] == want


def test_box_contains_cut_ellipse(ora):
    """Every pixel whose power (double precision) is >= the cut lies inside the clipped pixel box,
    so tiles are only a conservative accelerator; and the box is the per-axis extent of that
    ellipse rounded up to whole pixels (touching it within a pixel on at least one side)."""
    sc = scenes.make_scene(400, 0, log_scale_mean=-2.5)
    cams = scenes.make_cameras([(96, 80)])
    g = ora.geom32(sc, cams, 0)
    m, cov, _, _ = ora.project64(sc, cams, 0)
    ys, xs = np.mgrid[0:80, 0:96]
    px, py = xs + 0.5, ys + 0.5
    n_checked = 0
    for i in np.nonzero(g["participates"])[0]:
        det = cov[i, 0] * cov[i, 2] - cov[i, 1] ** 2
        a, b, c = cov[i, 2] / det, -cov[i, 1] / det, cov[i, 0] / det
        dx, dy = px - m[i, 0], py - m[i, 1]
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        cut = max(-4.5, -math.log(255.0 * float(sc.opacities[i])))
        inside = power >= cut + 1e-6
        if inside.any():
            yy, xx = np.nonzero(inside)
            assert xx.min() >= g["x0"][i] and xx.max() <= g["x1"][i]
            assert yy.min() >= g["y0"][i] and yy.max() <= g["y1"][i]
            n_checked += 1
        rx = math.ceil(math.sqrt(-2 * cut * cov[i, 0]) - 1e-5)
        ry = math.ceil(math.sqrt(-2 * cut * cov[i, 2]) - 1e-5)
        assert g["radius"][i] in (max(rx, ry), max(rx, ry) + 1)
    assert n_checked > 50


def test_transparent_gaussians_do_not_take_part(ora):
    """opacity < 1/255 can never give alpha >= 1/255: the cut ellipse is empty."""
    cam = _cam()
    for o, want in [(0.5 / 255, 0), (2.0 / 255, 1), (0.9, 1)]:
        sc = _one((0, 0, 0), (0.05,) * 3, (1, 0, 0, 0), opac=o)
        assert ora.geom32(sc, [cam], 0)[0]["participates"] == want


def test_cut_thresholds(ora):
    sc = scenes.make_scene(500, 0)
    cams = scenes.make_cameras([(128, 128)])
    g = ora.geom32(sc, cams, 0)
    p = g["participates"] == 1
    o = sc.opacities.astype(np.float64)
    expect_cut = np.maximum(-4.5, -np.log(255.0 * o))
    assert np.allclose(g["cut"][p], expect_cut[p], atol=3e-6)
    assert np.allclose(g["hi"][p], np.log(0.99 / o[p]), atol=3e-6)


def test_binning_invariants(ora):
    sc = scenes.make_scene(1500, 0, log_scale_mean=-3.0)
    cams = scenes.make_cameras([(70, 50), (33, 64), (64, 64)])
    tile = (16, 8)
    keys, vals, ranges = ora.binning(sc, cams, tile)
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)
    # ties broken by Gaussian index
    same = keys[1:] == keys[:-1]
    assert np.all(vals[1:][same] > vals[:-1][same])
    # every (Gaussian, covered tile) appears exactly once; brute-force overlap enumeration
    expect = set()
    for v in range(3):
        g = ora.geom32(sc, cams, v, tile)
        for i in np.nonzero(g["participates"])[0]:
            for ty in range(g["y0"][i] // tile[1], g["y1"][i] // tile[1] + 1):
                for tx in range(g["x0"][i] // tile[0], g["x1"][i] // tile[0] + 1):
                    tl = ty * ((cams[v].width + tile[0] - 1) // tile[0]) + tx
                    expect.add((v, tl, int(g["depth_bits"][i]), int(i)))
    got = set((int(k >> 48), int((k >> 32) & 0xFFFF), int(k & 0xFFFFFFFF), int(g_)) for k, g_ in zip(keys, vals))
    assert got == expect
    assert len(keys) == len(expect)
    # ranges partition the sorted array by (view, tile)
    tb = 0
    for v, c in enumerate(cams):
        nt = ((c.width + tile[0] - 1) // tile[0]) * ((c.height + tile[1] - 1) // tile[1])
        for tl in range(nt):
            a, b = ranges[tb + tl]
            sel = np.nonzero(((keys >> 48) == v) & (((keys >> 32) & 0xFFFF) == tl))[0]
            if len(sel) == 0:
                assert a == 0 and b == 0
            else:
                assert (a, b) == (sel[0], sel[-1] + 1)
        tb += nt
