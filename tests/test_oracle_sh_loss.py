"""Pins of the oracle's spherical harmonics and photometric losses.

SH: orthonormality by spherical quadrature, parity, the degree-0 constant, the
degree-1 closed forms, scipy's complex SH, and finite differences of the gradient.
Loss (Sec. 3; Sec. 5.1.2, Eqs. 7-10): SSIM(I, I) = 1, scipy's correlate for the
windowed moments, and finite differences of the image gradient."""
import math

import numpy as np
import pytest
import scipy.ndimage
import scipy.special

from paper_2506_12727_amd import scenes


def _dirs(n, seed=0):
    d = np.random.default_rng(seed).normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def test_sh_orthonormal_by_quadrature(ora):
    nt, nph = 24, 48
    xg, wg = np.polynomial.legendre.leggauss(nt)       # z = cos(theta)
    phis = (np.arange(nph) + 0.5) * 2 * math.pi / nph
    G = np.zeros((16, 16))
    for z, wz in zip(xg, wg):
        st = math.sqrt(1 - z * z)
        for ph in phis:
            Y, _ = ora.sh_basis(3, [st * math.cos(ph), st * math.sin(ph), z])
            G += np.outer(Y, Y) * wz * (2 * math.pi / nph)
    assert np.allclose(G, np.eye(16), atol=1e-12)


def test_sh_parity_and_low_orders(ora):
    c1 = math.sqrt(3 / (4 * math.pi))
    for d in _dirs(50):
        Y, _ = ora.sh_basis(3, d)
        Yn, _ = ora.sh_basis(3, -d)
        for l in range(4):
            sl = slice(l * l, (l + 1) * (l + 1))
            assert np.allclose(Yn[sl], (-1) ** l * Y[sl], atol=1e-14)
        assert abs(Y[0] - 0.5 / math.sqrt(math.pi)) < 1e-15
        # Condon-Shortley phase: (m=-1, 0, 1) = (-c1 y, c1 z, -c1 x)
        assert np.allclose(Y[1:4], [-c1 * d[1], c1 * d[2], -c1 * d[0]], atol=1e-14)


def test_sh_matches_scipy_complex_harmonics(ora):
    for d in _dirs(30, seed=3):
        theta = math.acos(d[2])               # polar
        phi = math.atan2(d[1], d[0])          # azimuth
        Y, _ = ora.sh_basis(3, d)
        for l in range(4):
            for m in range(-l, l + 1):
                c = scipy.special.sph_harm_y(l, abs(m), theta, phi)
                if m == 0:
                    want = c.real
                elif m > 0:
                    want = math.sqrt(2) * c.real
                else:
                    want = math.sqrt(2) * c.imag
                assert abs(Y[l * l + l + m] - want) < 1e-12, (l, m)


def test_sh_gradient_finite_differences(ora):
    h = 1e-6
    for d in _dirs(10, seed=7):
        _, dY = ora.sh_basis(3, d)
        P = np.eye(3) - np.outer(d, d)       # only the tangential part is defined on the sphere
        for k in range(3):
            e = P[:, k]
            dp = (d + h * e) / np.linalg.norm(d + h * e)
            dm = (d - h * e) / np.linalg.norm(d - h * e)
            fd = (ora.sh_basis(3, dp)[0] - ora.sh_basis(3, dm)[0]) / (2 * h)
            assert np.allclose(fd, dY @ (P @ e), atol=1e-7)


def test_degree0_colour(ora):
    sc = scenes.make_scene(50, 0)
    cams = scenes.make_cameras([(64, 64)])
    _, _, rgb, _ = ora.project64(sc, cams, 0)
    raw = sc.sh[:, 0, :].astype(np.float64) * (0.5 / math.sqrt(math.pi)) + 0.5
    assert np.allclose(rgb, np.maximum(raw, 0), atol=1e-12)


def _window():
    u = np.arange(11) - 5
    g = np.exp(-(u[:, None] ** 2 + u[None, :] ** 2) / (2 * 1.5 ** 2))
    return g / g.sum()


def test_ssim_map_vs_scipy_correlate(ora):
    rng = np.random.default_rng(1)
    a, b = rng.uniform(size=(23, 31)), rng.uniform(size=(23, 31))
    w = _window()
    f = lambda x: scipy.ndimage.correlate(x, w, mode="constant", cval=0.0)
    mu1, mu2 = f(a), f(b)
    s11, s22, s12 = f(a * a) - mu1 ** 2, f(b * b) - mu2 ** 2, f(a * b) - mu1 * mu2
    C1, C2 = 0.01 ** 2, 0.03 ** 2
    want = (2 * mu1 * mu2 + C1) * (2 * s12 + C2) / ((mu1 ** 2 + mu2 ** 2 + C1) * (s11 + s22 + C2))
    assert np.allclose(ora.ssim_map(a, b), want, atol=1e-13)


def test_ssim_identity_and_zero_gradient(ora):
    cams = scenes.make_cameras([(20, 17), (9, 12)])
    rng = np.random.default_rng(2)
    imgs = [rng.uniform(size=(3, c.height, c.width)) for c in cams]
    loss, grads = ora.loss(cams, imgs, imgs, 0.0, 1.0)
    assert abs(loss) < 1e-14
    assert max(np.abs(g).max() for g in grads) < 1e-14


def test_l1_gradient_is_sign_over_count(ora):
    cams = scenes.make_cameras([(20, 17), (9, 12)])
    rng = np.random.default_rng(3)
    imgs = [rng.uniform(size=(3, c.height, c.width)) for c in cams]
    tg = [rng.uniform(size=(3, c.height, c.width)) for c in cams]
    N = sum(3 * c.width * c.height for c in cams)
    loss, grads = ora.loss(cams, imgs, tg, 1.0, 0.0)
    assert abs(loss - sum(np.abs(a - b).sum() for a, b in zip(imgs, tg)) / N) < 1e-14
    for g, a, b in zip(grads, imgs, tg):
        assert np.array_equal(g, np.sign(a - b) / N)


def test_dssim_gradient_finite_differences(ora):
    cams = scenes.make_cameras([(14, 11), (9, 13)])
    rng = np.random.default_rng(4)
    imgs = [rng.uniform(size=(3, c.height, c.width)) for c in cams]
    tg = [rng.uniform(size=(3, c.height, c.width)) for c in cams]
    _, grads = ora.loss(cams, imgs, tg, 0.0, 1.0)
    h = 1e-6
    for _ in range(25):
        v = int(rng.integers(2))
        idx = tuple(int(rng.integers(n)) for n in imgs[v].shape)
        ip = [a.copy() for a in imgs]; ip[v][idx] += h
        im = [a.copy() for a in imgs]; im[v][idx] -= h
        fd = (ora.loss(cams, ip, tg, 0.0, 1.0)[0] - ora.loss(cams, im, tg, 0.0, 1.0)[0]) / (2 * h)
        assert abs(fd - grads[v][idx]) < 1e-8 * max(1.0, abs(fd)) + 1e-4 * abs(fd)
