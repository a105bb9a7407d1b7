"""Pins of the pose-initialisation oracle (oracle/tracking.py): exact recovery from
noise-free correspondences, outlier rejection, the optimality of the refined pose and the
se(3) exponential."""
import numpy as np
import pytest

from oracle import tracking as TK
from paper_2507_03737_amd import scenes

K = (572.0, 572.0, 480.0, 320.0)


def _problem(n, seed, outliers=0.0, noise=0.0):
    rng = np.random.default_rng(seed)
    T = scenes.perturb_pose(np.concatenate([np.eye(3), np.zeros((3, 1))], 1).reshape(-1), 8.0, 1.0, seed)
    T = np.asarray(T, float).reshape(3, 4)
    U, _, Vt = np.linalg.svd(T[:, :3])                                  # exact rotation in float64
    T[:, :3] = U @ Vt
    z = rng.uniform(3.0, 40.0, n)
    u = rng.uniform(0, 960, n)
    v = rng.uniform(0, 640, n)
    Xb = np.stack([(u - K[2]) / K[0] * z, (v - K[3]) / K[1] * z, z])     # points in frame B
    X = T[:, :3].T @ (Xb - T[:, 3:4])                                     # the same points in frame A
    uv = np.stack([u, v]) + rng.normal(0.0, noise, (2, n))
    bad = rng.random(n) < outliers
    ang = rng.uniform(0, 2 * np.pi, bad.sum())
    off = rng.uniform(20.0, 200.0, bad.sum())              # far from the true reprojection
    uv[:, bad] += off * np.stack([np.cos(ang), np.sin(ang)])
    samples = rng.integers(0, n, (256, 6))
    return X, uv, T, bad, samples


def test_dlt_exact_on_noise_free_points():
    X, uv, T, _, _ = _problem(6, 0)
    P, gap = TK.dlt_pose(X, uv, K)
    np.testing.assert_allclose(P, T, atol=1e-9)
    assert gap > 1e-8


def test_ransac_recovers_pose_and_outliers():
    X, uv, T, bad, samples = _problem(2000, 1, outliers=0.3)
    r = TK.pnp_ransac(X, uv, K, samples, thr=2.0)
    np.testing.assert_allclose(r["T"], T, atol=1e-9)
    assert np.array_equal(r["inliers"], ~bad)


def test_refined_pose_is_stationary_and_close():
    X, uv, T, bad, samples = _problem(1500, 2, outliers=0.2, noise=0.5)
    r = TK.pnp_ransac(X, uv, K, samples, thr=3.0, iters=15)
    ok = r["inliers"]
    # Stationarity: a small left perturbation in any direction does not decrease the cost.
    def cost(Tp):
        res, _ = TK.reproj(Tp, X[:, ok], uv[:, ok], K)
        return (res ** 2).sum()
    c0 = cost(r["T"])
    for k in range(6):
        for sgn in (1.0, -1.0):
            xi = np.zeros(6)
            xi[k] = sgn * 1e-5
            assert cost(TK.compose(TK.se3_exp(xi), r["T"])) >= c0 - 1e-9 * c0
    R_err = r["T"][:, :3] @ T[:, :3].T
    assert np.degrees(np.arccos(np.clip((np.trace(R_err) - 1) / 2, -1, 1))) < 0.05
    assert np.linalg.norm(r["T"][:, 3] - T[:, 3]) < 0.02


def test_se3_exp_matches_rodrigues_and_composes():
    phi = np.array([0.3, -0.2, 0.5])
    th = np.linalg.norm(phi)
    k = phi / th
    Kx = TK._hat(k)
    R = np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx
    E = TK.se3_exp(np.concatenate([[0.0, 0.0, 0.0], phi]))
    np.testing.assert_allclose(E[:, :3], R, atol=1e-14)
    E2 = TK.se3_exp(np.concatenate([[1.0, 2.0, 3.0], [0.0, 0.0, 0.0]]))
    np.testing.assert_allclose(E2, np.concatenate([np.eye(3), [[1.0], [2.0], [3.0]]], 1), atol=1e-15)
