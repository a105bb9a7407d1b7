"""FP64 oracle for the pose initialisation of the tracking front end (numpy).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and never by the product path.

Sec. 3.2.1 (Eq. 6-9): 2D-3D correspondences between the rendered pointmap of the
adjacent keyframe (3D points X in that keyframe's camera frame) and pixels u of the new
frame give the relative pose T_rel (X -> camera frame of the new frame) by RANSAC and
PnP; the new pose is T_n = T_rel T_ak.  The paper names RANSAC and a PnP solver but not
their inner steps; this oracle (and the library) use:

* hypotheses: the linear six-point PnP (DLT) on a caller-given sample of 6
  correspondences, with the 3D points translated to their centroid and scaled to mean
  distance sqrt(3); the 12-vector is the eigenvector of A^T A with the smallest
  eigenvalue; its sign makes det(M) > 0 for M the left 3x3 block; R = U V^T from the SVD
  M = U S V^T, lambda = mean(S), t = p_4 / lambda (after undoing the normalisation);
* score: the number of correspondences whose reprojection error |pi(R X + t) - u| (pixels)
  is below the threshold and whose depth (R X + t)_z is positive;
* best hypothesis: the highest score, ties to the lowest hypothesis index;
* refinement: Gauss-Newton on the sum of squared reprojection errors of the inliers,
  with the pose perturbed on the left, T <- Exp(xi) T, xi = (rho, phi); the inlier set is
  re-selected with the refined pose and the refinement repeated, ``rounds`` times;
  each Gauss-Newton step solves (J^T J + 1e-9 trace(J^T J)/6 I) xi = -J^T r.
"""
from __future__ import annotations

import numpy as np


def _hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def se3_exp(xi):
    """Exp of xi = (rho, phi) as a 3x4 [R | t] (Rodrigues; V for the translation)."""
    rho, phi = np.asarray(xi[:3], float), np.asarray(xi[3:], float)
    th = np.linalg.norm(phi)
    K = _hat(phi)
    if th < 1e-12:
        R = np.eye(3) + K
        V = np.eye(3) + 0.5 * K
    else:
        a, b, c = np.sin(th) / th, (1 - np.cos(th)) / th ** 2, (th - np.sin(th)) / th ** 3
        R = np.eye(3) + a * K + b * K @ K
        V = np.eye(3) + b * K + c * K @ K
    return np.concatenate([R, (V @ rho)[:, None]], axis=1)


def compose(A, B):
    """[R_a | t_a] [R_b | t_b] as 3x4."""
    A, B = np.asarray(A, float).reshape(3, 4), np.asarray(B, float).reshape(3, 4)
    return np.concatenate([A[:, :3] @ B[:, :3], (A[:, :3] @ B[:, 3] + A[:, 3])[:, None]], axis=1)


def normalised(uv, K):
    fx, fy, cx, cy = K
    return np.stack([(uv[0] - cx) / fx, (uv[1] - cy) / fy])


def dlt_pose(X, uv, K):
    """Linear PnP on >= 6 correspondences: X [3][m], uv [2][m] -> (3x4 pose, eigenvalue gap)."""
    X = np.asarray(X, float)
    x = normalised(np.asarray(uv, float), K)
    c = X.mean(axis=1)
    d = np.sqrt(((X - c[:, None]) ** 2).sum(axis=0)).mean()
    s = np.sqrt(3.0) / d if d > 0 else 1.0
    Xn = s * (X - c[:, None])
    m = X.shape[1]
    A = np.zeros((2 * m, 12))
    for k in range(m):
        Xh = np.append(Xn[:, k], 1.0)
        A[2 * k, 0:4] = Xh
        A[2 * k, 8:12] = -x[0, k] * Xh
        A[2 * k + 1, 4:8] = Xh
        A[2 * k + 1, 8:12] = -x[1, k] * Xh
    w, V = np.linalg.eigh(A.T @ A)
    p = V[:, 0]
    Pn = p.reshape(3, 4)
    # Undo the normalisation: P = Pn [[s I, -s c], [0, 1]].
    M = s * Pn[:, :3]
    p4 = Pn[:, 3] - s * Pn[:, :3] @ c
    if np.linalg.det(M) < 0:
        M, p4 = -M, -p4
    U, S, Vt = np.linalg.svd(M)
    R = U @ Vt
    lam = S.mean()
    t = p4 / lam
    gap = (w[1] - w[0]) / max(w[-1], 1e-300)
    return np.concatenate([R, t[:, None]], axis=1), gap


def reproj(T, X, uv, K):
    """(pixel residuals [2][n], camera depths [n]) of X under pose T."""
    fx, fy, cx, cy = K
    T = np.asarray(T, float).reshape(3, 4)
    Y = T[:, :3] @ X + T[:, 3:4]
    z = Y[2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = fx * Y[0] / z + cx
        v = fy * Y[1] / z + cy
    return np.stack([u - uv[0], v - uv[1]]), z


def inliers(T, X, uv, K, thr):
    r, z = reproj(T, X, uv, K)
    e = np.sqrt((r ** 2).sum(axis=0))
    ok = (z > 0) & (e < thr)
    with np.errstate(invalid="ignore"):
        margin = np.abs(e - thr) / thr
    return ok, np.where(z > 0, margin, np.inf)


def refine(T, X, uv, K, iters=10):
    """Gauss-Newton on sum |pi(R X + t) - u|^2 with T <- Exp(xi) T."""
    fx, fy = K[0], K[1]
    T = np.asarray(T, float).reshape(3, 4)
    for _ in range(iters):
        Y = T[:, :3] @ X + T[:, 3:4]
        r, _ = reproj(T, X, uv, K)
        x, y, z = Y
        iz = 1.0 / z
        # d pi / d Y, then d Y / d xi = [I | -[Y]x].
        Ju = np.stack([fx * iz, np.zeros_like(z), -fx * x * iz * iz])
        Jv = np.stack([np.zeros_like(z), fy * iz, -fy * y * iz * iz])
        H = np.zeros((6, 6))
        g = np.zeros(6)
        for Jp, rr in ((Ju, r[0]), (Jv, r[1])):
            # d Y / d phi = -[Y]x, so the rotation block is Y x Jp.
            Jrot = np.stack([y * Jp[2] - z * Jp[1], z * Jp[0] - x * Jp[2], x * Jp[1] - y * Jp[0]])
            J = np.concatenate([Jp, Jrot])            # [6][n]
            H += J @ J.T
            g += J @ rr
        H += 1e-9 * np.trace(H) / 6.0 * np.eye(6)
        xi = -np.linalg.solve(H, g)
        T = compose(se3_exp(xi), T)
    return T


def pnp_ransac(X, uv, K, samples, thr=2.0, iters=10, rounds=2):
    """RANSAC over the given samples [H][6] of indices, then refinement.

    X [3][n] (frame A), uv [2][n] (pixels of frame B), K = (fx, fy, cx, cy).  Returns a dict
    with ``T`` (3x4, A -> B), ``inliers`` (mask), ``best`` (hypothesis index), ``scores``,
    ``gaps`` (eigenvalue gaps of the hypotheses) and ``margin`` (the smallest relative
    distance of a final inlier decision from the threshold)."""
    X = np.asarray(X, float)
    uv = np.asarray(uv, float)
    samples = np.asarray(samples)
    scores = np.zeros(len(samples), dtype=np.int64)
    gaps = np.zeros(len(samples))
    poses = []
    for h, idx in enumerate(samples):
        T, gaps[h] = dlt_pose(X[:, idx], uv[:, idx], K)
        poses.append(T)
        scores[h] = int(inliers(T, X, uv, K, thr)[0].sum())
    best = int(np.argmax(scores))                        # first maximum
    T = poses[best]
    ok = inliers(T, X, uv, K, thr)[0]
    for _ in range(rounds):
        if ok.sum() >= 6:
            T = refine(T, X[:, ok], uv[:, ok], K, iters)
        ok, margin = inliers(T, X, uv, K, thr)
    ok, margin = inliers(T, X, uv, K, thr)
    return {"T": T, "inliers": ok, "best": best, "scores": scores, "gaps": gaps,
            "margin": float(margin.min()) if margin.size else np.inf}
