"""Seeded synthetic inputs shared by the HIP path's tests, the benchmark and the oracle's tests.

This module only draws numbers: Gaussian parameters, cameras, poses and upstream
gradients, sampled in float64 with numpy's PCG64 and cast to float32.  It holds
none of the rasterizer's arithmetic (no projection, compositing or gradients), so
the oracle and the GPU path can both consume it without sharing method code.

Workloads (the paper measures on Waymo / KITTI / DL3DV sequences with MASt3R
priors, Sec. 4.1; none of that data is available, so these seeded scenes stand in
for it with the resolutions, window size (|W| = 8, Supp. S2.1) and outdoor
structure of those sequences):

* ``c0``  2,000 Gaussians, one 160x120 view, depth U[2, 20] m, screen-uniform.
* ``c1``  300k Gaussians, one 1216x352 view, outdoor street layout.
* ``c2``  500k Gaussians, one 960x640 view (tracking), same layout.
* ``c3``  1M Gaussians, 8 keyframes of uneven size along a driving trajectory.
* ``c4``  3M Gaussians, 16 keyframes of 1920x1080.

Parameter layout matches the library's: planar SoA ``means[3][N]``,
``log_scales[3][N]``, ``quats[4][N]`` (w, x, y, z), ``opacity_logit[N]``,
``rgb[3][N]``; poses ``T_cw[V][12]`` (world->camera, row-major 3x4, OpenCV axes).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

__all__ = [
    "Camera", "Scene", "make_scene", "upstream_grads", "perturb_pose",
    "rotation_about_axis", "CONFIG_NAMES", "street_pointmap", "noisy_prior",
]

CONFIG_NAMES = ("c0", "c1", "c2", "c3", "c4")

# 80 degree horizontal field of view for the outdoor configurations: fx = W / (2 tan 40deg).
_TAN40 = math.tan(math.radians(40.0))


@dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    @staticmethod
    def fov80(width: int, height: int, fx: float | None = None) -> "Camera":
        f = width / (2.0 * _TAN40) if fx is None else fx
        return Camera(width, height, float(np.float32(f)), float(np.float32(f)),
                      width / 2.0, height / 2.0)


@dataclass
class Scene:
    name: str
    means: np.ndarray          # float32 [3][N]
    log_scales: np.ndarray     # float32 [3][N]
    quats: np.ndarray          # float32 [4][N]
    opacity_logit: np.ndarray  # float32 [N]
    rgb: np.ndarray            # float32 [3][N]
    cams: List[Camera]
    T_cw: np.ndarray           # float32 [V][12]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def n_views(self) -> int:
        return len(self.cams)

    def params(self):
        return (self.means, self.log_scales, self.quats, self.opacity_logit, self.rgb)

    def subset(self, n: int) -> "Scene":
        """First ``n`` Gaussians (the draws are i.i.d., so this is an unbiased sub-sample)."""
        return Scene(self.name, self.means[:, :n].copy(), self.log_scales[:, :n].copy(),
                     self.quats[:, :n].copy(), self.opacity_logit[:n].copy(),
                     self.rgb[:, :n].copy(), list(self.cams), self.T_cw.copy(), dict(self.meta))


def rotation_about_axis(axis, angle: float) -> np.ndarray:
    """Rodrigues rotation matrix (float64) for a unit ``axis`` and ``angle`` in radians."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + math.sin(angle) * K + (1.0 - math.cos(angle)) * (K @ K)


def _pose_row(R_cw: np.ndarray, t_cw: np.ndarray) -> np.ndarray:
    return np.concatenate([np.concatenate([R_cw, t_cw[:, None]], axis=1).reshape(-1)])


def _random_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _loguniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def _street_points(rng, n, z_lo, z_hi, tan_half_fov):
    """Camera-frame centres of an outdoor street: 70% ground plane, 30% box facades.

    Every point draws its depth log-uniformly in [z_lo, z_hi].  Ground points sit on
    y = 1.6 m (camera 1.6 m above the road, y pointing down) with lateral position
    inside the view cone widened by 1.2.  Facade points belong to one of two rows of
    boxes along the street (x < 0 and x > 0).  Each row is a chain of segments of
    length U[5, 20] m along z; a segment has a lateral offset U[4, 12] m and a
    height U[4, 15] m.  A facade point lies on the street-facing wall of the
    segment containing its depth (x = +-offset) or, with probability 0.2, on the
    segment's front face (z = segment start, x = +-(offset + U[0, 4] m)); its
    height is y ~ U[1.6 - h, 1.6].
    """
    z = _loguniform(rng, z_lo, z_hi, n)
    pts = np.empty((3, n))
    ground = rng.uniform(size=n) < 0.7
    ng = int(ground.sum())
    pts[0, ground] = rng.uniform(-1.2, 1.2, ng) * z[ground] * tan_half_fov
    pts[1, ground] = 1.6
    pts[2, ground] = z[ground]

    fac = ~ground
    nf = int(fac.sum())
    zf = z[fac]
    side = np.where(rng.uniform(size=nf) < 0.5, -1.0, 1.0)
    x = np.empty(nf)
    y = np.empty(nf)
    zz = zf.copy()
    for s in (-1.0, 1.0):
        # Chain of segments covering [z_lo, z_hi] on this side of the street.
        starts, offs, hts = [], [], []
        cur = z_lo
        while cur < z_hi:
            starts.append(cur)
            offs.append(rng.uniform(4.0, 12.0))
            hts.append(rng.uniform(4.0, 15.0))
            cur += rng.uniform(5.0, 20.0)
        starts = np.array(starts)
        offs = np.array(offs)
        hts = np.array(hts)
        sel = side == s
        idx = np.clip(np.searchsorted(starts, zf[sel], side="right") - 1, 0, len(starts) - 1)
        front = rng.uniform(size=int(sel.sum())) < 0.2
        xo = offs[idx] + np.where(front, rng.uniform(0.0, 4.0, int(sel.sum())), 0.0)
        x[sel] = s * xo
        zz_sel = np.where(front, starts[idx], zf[sel])
        zz[sel] = zz_sel
        y[sel] = 1.6 - rng.uniform(0.0, 1.0, int(sel.sum())) * hts[idx]
    pts[0, fac] = x
    pts[1, fac] = y
    pts[2, fac] = zz
    return pts


def _attributes(rng, n, ls_mu, ls_sd, logit_mu, logit_sd):
    log_scales = rng.normal(ls_mu, ls_sd, (3, n))
    quats = _random_quats(rng, n)
    logit = rng.normal(logit_mu, logit_sd, n)
    rgb = rng.uniform(0.0, 1.0, (3, n))
    return log_scales, quats, logit, rgb


def _trajectory(rng, n_views, spacing, yaw_deg):
    """Keyframe poses along +z with small random yaw; returns (R_wc, C) lists."""
    poses = []
    for k in range(n_views):
        yaw = math.radians(rng.uniform(-yaw_deg, yaw_deg))
        R_wc = rotation_about_axis([0.0, 1.0, 0.0], yaw)
        C = np.array([0.0, 0.0, spacing * k])
        poses.append((R_wc, C))
    return poses


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def make_scene(name: str, seed: int | None = None, n: int | None = None) -> Scene:
    """Build configuration ``name`` (c0..c4).  ``seed`` defaults to the config index."""
    k = CONFIG_NAMES.index(name)
    rng = np.random.default_rng(k if seed is None else seed)

    if name == "c0":
        n = 2000 if n is None else n
        cam = Camera(160, 120, 128.0, 128.0, 80.0, 60.0)
        z = rng.uniform(2.0, 20.0, n)
        u = rng.uniform(0.0, cam.width, n)
        v = rng.uniform(0.0, cam.height, n)
        means = np.stack([(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z])
        ls, q, lo, rgb = _attributes(rng, n, -2.5, 0.5, 0.0, 1.0)
        cams = [cam]
        T = np.array([_pose_row(np.eye(3), np.zeros(3))])
    elif name in ("c1", "c2"):
        if name == "c1":
            n = 300_000 if n is None else n
            cam = Camera.fov80(1216, 352)
        else:
            n = 500_000 if n is None else n
            cam = Camera.fov80(960, 640)
        means = _street_points(rng, n, 1.0, 80.0, _TAN40)
        ls, q, lo, rgb = _attributes(rng, n, -3.0, 0.7, 0.5, 1.5)
        cams = [cam]
        T = np.array([_pose_row(np.eye(3), np.zeros(3))])
    elif name in ("c3", "c4"):
        if name == "c3":
            n = 1_000_000 if n is None else n
            cams = ([Camera.fov80(960, 640)] * 3 + [Camera.fov80(1216, 352)] * 3
                    + [Camera.fov80(640, 480)] * 2)
            poses = _trajectory(rng, 8, 1.5, 5.0)
            z_lo, z_hi, ls_mu, ls_sd = 1.0, 80.0, -3.0, 0.7
        else:
            n = 3_000_000 if n is None else n
            cams = [Camera(1920, 1080, 1144.0, 1144.0, 960.0, 540.0)] * 16
            poses = _trajectory(rng, 16, 1.0, 5.0)
            z_lo, z_hi, ls_mu, ls_sd = 0.5, 120.0, -3.5, 0.8
        owner = rng.integers(0, len(cams), n)
        local = _street_points(rng, n, z_lo, z_hi, _TAN40)
        means = np.empty((3, n))
        for v, (R_wc, C) in enumerate(poses):
            sel = owner == v
            means[:, sel] = R_wc @ local[:, sel] + C[:, None]
        ls, q, lo, rgb = _attributes(rng, n, ls_mu, ls_sd, 0.5, 1.5)
        T = np.array([_pose_row(R_wc.T, -R_wc.T @ C) for (R_wc, C) in poses])
    else:  # pragma: no cover - guarded by CONFIG_NAMES.index
        raise ValueError(name)

    return Scene(name, _f32(means), _f32(ls), _f32(q), _f32(lo), _f32(rgb), cams, _f32(T),
                 meta={"seed": k if seed is None else seed})


def upstream_grads(scene: Scene, seed: int = 1000, alpha: bool = False):
    """Per-view upstream gradients N(0, 1) for RGB, depth and pointmap (alpha 0 unless asked).

    Returns a list of dicts with float32 planar arrays rgb[3][H][W], depth[H][W],
    alpha[H][W], pointmap[3][H][W].
    """
    rng = np.random.default_rng(seed)
    out = []
    for cam in scene.cams:
        H, W = cam.height, cam.width
        out.append({
            "rgb": _f32(rng.standard_normal((3, H, W))),
            "depth": _f32(rng.standard_normal((H, W))),
            "alpha": _f32(rng.standard_normal((H, W)) if alpha else np.zeros((H, W))),
            "pointmap": _f32(rng.standard_normal((3, H, W))),
        })
    return out


def perturb_pose(T_row: np.ndarray, deg: float, meters: float, seed: int) -> np.ndarray:
    """Left-multiply a 3x4 world->camera pose by a rotation of ``deg`` degrees about a
    random axis and a translation of ``meters`` in a random direction (float32 [12])."""
    rng = np.random.default_rng(seed)
    axis = rng.standard_normal(3)
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    R_d = rotation_about_axis(axis, math.radians(deg))
    T = np.asarray(T_row, dtype=np.float64).reshape(3, 4)
    R = R_d @ T[:, :3]
    t = R_d @ T[:, 3] + meters * d
    return _f32(np.concatenate([R, t[:, None]], axis=1).reshape(-1))


def street_pointmap(cam: Camera, seed: int) -> np.ndarray:
    """Camera-frame pointmap [3][H][W] (float32) of a synthetic street view: a ground plane
    1.6 m below the camera up to 80 m, walls 6-10 m to either side and a far backdrop,
    with centimetre-scale surface roughness.  Stands in for a rendered pointmap."""
    rng = np.random.default_rng(seed)
    H, W = cam.height, cam.width
    jj, ii = np.mgrid[0:H, 0:W].astype(np.float64)
    rx, ry = (ii - cam.cx) / cam.fx, (jj - cam.cy) / cam.fy
    z = np.full((H, W), 80.0)
    ground = ry > 1e-3
    z[ground] = np.minimum(80.0, 1.6 / ry[ground])
    for side, off in ((-1.0, rng.uniform(6.0, 10.0)), (1.0, rng.uniform(6.0, 10.0))):
        hit = side * rx > 1e-3
        zw = off / np.abs(rx[hit])
        z[hit] = np.minimum(z[hit], zw)
    z *= 1.0 + rng.normal(0.0, 0.003, (H, W))
    return _f32(np.stack([rx * z, ry * z, z]))


def noisy_prior(Xr: np.ndarray, scale: float, seed: int, noise: float = 0.01, patch: int = 10,
                outlier_patches: float = 0.1, outlier_pixels: float = 0.01) -> np.ndarray:
    """A prior pointmap at another scale: Xr / scale with relative noise, a fraction of whole
    patches at an unrelated scale and a fraction of isolated pixels pushed far off."""
    rng = np.random.default_rng(seed)
    _, H, W = Xr.shape
    Xp = Xr.astype(np.float64) / scale * (1.0 + rng.normal(0.0, noise, (1, H, W)))
    nph, npw = -(-H // patch), -(-W // patch)
    bad = rng.random((nph, npw)) < outlier_patches
    f = np.repeat(np.repeat(np.where(bad, rng.uniform(0.3, 3.0, (nph, npw)), 1.0), patch, 0), patch, 1)[:H, :W]
    Xp *= f[None]
    px = rng.random((H, W)) < outlier_pixels
    Xp[:, px] *= rng.uniform(2.0, 5.0, px.sum())[None]
    return _f32(Xp)
