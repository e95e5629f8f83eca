"""The oracle's multi-view adaptive density control (Sec. 5.2.2): split on mean E1, clone on mean
E2, prune on opacity; pinned by hand-built cases and by the children's sample statistics."""
import numpy as np

import oracle


def _gaussians(n, big):
    rng = np.random.default_rng(0)
    means = rng.uniform(-1, 1, (n, 3))
    scales = np.where(big[:, None], 0.05, 0.002) * rng.uniform(0.5, 1.0, (n, 3))
    quats = rng.normal(size=(n, 4))
    opac = rng.uniform(0.2, 0.9, n)
    sh = rng.normal(size=(n, 4, 3))
    return means, scales, quats, opac, sh


def test_each_rule_on_hand_built_cases():
    big = np.array([True, True, False, False, False, True])
    means, scales, quats, opac, sh = _gaussians(6, big)
    opac[4] = 0.001                                   # pruned
    e1 = np.array([10.0, 0.1, 10.0, 0.1, 10.0, 10.0])
    e2 = np.array([10.0, 0.1, 0.1, 10.0, 10.0, 10.0])
    count = np.array([2, 2, 2, 2, 2, 0])             # g = 5 never seen: kept
    normals = np.zeros((6, 2, 3))
    nm, ns, nq, no, nsh, src = oracle.densify(means, scales, quats, opac, sh, e1, e2, count, normals,
                                              split_threshold=1.0, clone_threshold=1.0, dense_scale=0.01,
                                              min_opacity=0.005)
    # g0 big, high E1 -> two children; g1 big, low -> kept; g2 small, high E1 only -> kept;
    # g3 small, high E2 -> cloned; g4 pruned; g5 no views -> kept
    assert list(src) == [0, 0, 1, 2, 3, 3, 5]
    assert np.allclose(ns[0], scales[0] / 1.6) and np.allclose(ns[1], scales[0] / 1.6)
    assert np.allclose(nm[0], means[0]) and np.allclose(nm[1], means[0])   # z = 0: at the mean
    assert np.allclose(ns[4], scales[3]) and np.allclose(ns[5], scales[3])
    assert np.allclose(nm[4], means[3]) and np.allclose(nm[5], means[3])
    for i, g in enumerate(src):
        assert np.allclose(nq[i], quats[g]) and no[i] == opac[g] and np.allclose(nsh[i], sh[g])


def test_split_children_are_samples_of_the_parent():
    """Children of one parent drawn with many normals have the parent's mean and covariance
    R diag(s^2) R^T."""
    n = 4000
    big = np.ones(n, bool)
    means, scales, quats, opac, sh = _gaussians(n, big)
    means[:] = means[0]; scales[:] = scales[0] * np.array([1.0, 0.5, 2.0]); quats[:] = quats[0]
    rng = np.random.default_rng(1)
    normals = rng.normal(size=(n, 2, 3))
    nm, ns, *_ = oracle.densify(means, scales, quats, opac, sh, np.full(n, 10.0), np.zeros(n), np.ones(n, int),
                                normals, 1.0, 1.0, 0.0, 0.0)
    assert len(nm) == 2 * n
    q = quats[0] / np.linalg.norm(quats[0])
    from scipy.spatial.transform import Rotation
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
    cov = R @ np.diag(scales[0] ** 2) @ R.T
    d = nm - means[0]
    assert np.allclose(d.mean(0), 0.0, atol=4 * scales[0].max() / np.sqrt(2 * n))
    assert np.allclose(np.cov(d.T), cov, rtol=0.08, atol=0.08 * np.abs(cov).max())


def test_thresholds_are_strict_and_counts_divide():
    big = np.array([True, False])
    means, scales, quats, opac, sh = _gaussians(2, big)
    e = np.array([4.0, 4.0])
    count = np.array([4, 4])      # mean exactly 1.0 = threshold: nothing happens
    out = oracle.densify(means, scales, quats, opac, sh, e, e, count, np.zeros((2, 2, 3)), 1.0, 1.0, 0.01, 0.0)
    assert list(out[-1]) == [0, 1]
    count = np.array([3, 3])      # mean 4/3 > 1: split g0, clone g1
    out = oracle.densify(means, scales, quats, opac, sh, e, e, count, np.zeros((2, 2, 3)), 1.0, 1.0, 0.01, 0.0)
    assert list(out[-1]) == [0, 0, 1, 1]
