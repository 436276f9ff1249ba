"""Pins of the oracle's point-to-point ICP (Sec. 2.3 fine registration):
nearest neighbours against a k-d tree, the least-squares rigid update
against exact correspondences, rejection beyond the distance bound, and
recovery of a known rigid motion between two clouds of one surface."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle


def rot(ax, ay, az):
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def surface(n, seed):
    """Points of a smooth terrain patch z = f(x, y) (a cloud from one view)."""
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-10.0, 10.0, size=(n, 2))
    z = 2.0 * np.sin(0.4 * xy[:, 0]) * np.cos(0.3 * xy[:, 1]) + 0.05 * xy[:, 0] ** 2
    return np.column_stack([xy, z]).astype(np.float32)


def test_nearest_neighbours_match_kdtree():
    rng = np.random.default_rng(0)
    src = rng.uniform(-5, 5, size=(500, 3)).astype(np.float32)
    dst = rng.uniform(-5, 5, size=(700, 3)).astype(np.float32)
    moved, corr, d2 = oracle.icp_correspond(src, dst, np.eye(3), np.zeros(3), dmax=1.0)
    dist, idx = cKDTree(dst.astype(np.float64)).query(src.astype(np.float64))
    near = dist <= 1.0 - 1e-5
    far = dist > 1.0 + 1e-5
    np.testing.assert_array_equal(corr[near], idx[near])
    assert (corr[far] == -1).all()
    np.testing.assert_allclose(np.sqrt(d2[near]), dist[near], rtol=1e-5)
    np.testing.assert_array_equal(moved, src)


def test_rigid_update_exact_correspondences():
    p = surface(300, 1).astype(np.float64)
    R, T = rot(0.3, -0.2, 0.9), np.array([1.0, -2.0, 0.5])
    q = p @ R.T + T
    Re, Te = oracle.kabsch(p, q)
    np.testing.assert_allclose(Re, R, atol=1e-12)
    np.testing.assert_allclose(Te, T, atol=1e-11)
    # A proper rotation even for a planar point set.
    flat = p.copy()
    flat[:, 2] = 0.0
    Rf, _ = oracle.kabsch(flat, flat @ R.T)
    np.testing.assert_allclose(Rf @ Rf.T, np.eye(3), atol=1e-12)
    assert abs(np.linalg.det(Rf) - 1.0) < 1e-12


def test_icp_recovers_rigid_motion():
    src = surface(3000, 2)
    R, T = rot(0.02, -0.03, 0.05), np.array([0.4, -0.3, 0.2])
    dst = (src.astype(np.float64) @ R.T + T).astype(np.float32)
    Re, Te, rms, npairs, _ = oracle.icp(src, dst, np.eye(3), np.zeros(3), iters=40, dmax=2.0)
    np.testing.assert_allclose(Re, R, atol=2e-5)
    np.testing.assert_allclose(Te, T, atol=2e-4)
    assert rms[-1] < 1e-3 and rms[0] > 0.1
    assert npairs[-1] == len(src)


def test_rejection_beyond_bound():
    src = np.array([[0, 0, 0], [10, 0, 0]], dtype=np.float32)
    dst = np.array([[0.5, 0, 0], [3, 0, 0]], dtype=np.float32)
    _, corr, d2 = oracle.icp_correspond(src, dst, np.eye(3), np.zeros(3), dmax=1.0)
    assert list(corr) == [0, -1]
    assert d2[0] == np.float32(0.25)
