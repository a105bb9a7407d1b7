"""Helpers for the GPU-vs-oracle parity tests.

Tolerances (stated by the method's accuracy targets, applied per view and channel):

* images: |x - r| <= 1e-4 (|r| + 1e-3 max|r|) on every pixel the oracle does not flag as
  ambiguous (a float32 decision within rounding of a threshold); for the pointmap, a
  3-vector per pixel, |r| is the norm of the pixel's point (a coordinate that nearly
  cancels, such as x on the principal column, carries the rounding of terms of the
  point's own size);
* gradients, per tensor: ||g - r||_2 / ||r||_2 <= 2e-3, and |g - r| <= 2e-3 (|r| + rms(r))
  for at least 99.99% of the elements.
"""
from __future__ import annotations

import math
import sys

import numpy as np

IMG_RTOL = 1e-4
GRAD_RTOL = 2e-3


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(scene, torch):
    params = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in scene.params()]
    T = torch.from_numpy(np.ascontiguousarray(scene.T_cw)).cuda()
    return params, T


def check_image(name, got, ref, ok_mask, vector=False):
    """got, ref: [..., H, W] arrays; ok_mask: [H, W] bool of pixels to compare.  With
    vector=True the leading axis holds the components of one vector per pixel and the
    relative part of the tolerance uses the vector's norm."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.abs(ref).max() if ref.size else 0.0
    mag = np.sqrt((ref ** 2).sum(axis=0, keepdims=True)) if vector else np.abs(ref)
    tol = IMG_RTOL * (mag + 1e-3 * scale)
    bad = (np.abs(got - ref) > tol) & ok_mask
    if bad.any():
        idx = np.argwhere(bad)[:5]
        det = [(tuple(i), float(got[tuple(i)]), float(ref[tuple(i)])) for i in idx]
        raise AssertionError(f"{name}: {int(bad.sum())} pixels outside tolerance, e.g. {det}")


def check_grad(name, got, ref, frac=0.9999):
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    ref = np.asarray(ref, dtype=np.float64).reshape(-1)
    nr = np.linalg.norm(ref)
    rel = np.linalg.norm(got - ref) / nr if nr > 0 else np.linalg.norm(got)
    rms = math.sqrt(float(np.mean(ref ** 2))) if ref.size else 0.0
    bad = np.abs(got - ref) > GRAD_RTOL * (np.abs(ref) + rms)
    ok_frac = 1.0 - bad.mean() if ref.size else 1.0
    if not (rel <= GRAD_RTOL and ok_frac >= frac):
        idx = np.argwhere(bad).reshape(-1)[:5]
        raise AssertionError(f"{name}: rel L2 {rel:.3e}, elementwise ok {ok_frac:.6f}; e.g. "
                             f"{[(int(i), float(got[i]), float(ref[i])) for i in idx]}")
    return rel


def oracle_view_images(O, params_o, cam, T12, S, pixels=None, proj=None):
    """Oracle render of a full view or of the given pixels (returns per-pixel dict)."""
    view = O.make_view(cam, T12)
    pix = O.full_pixels(cam) if pixels is None else pixels
    return O.render(params_o, view, S, pix, proj=proj), pix


def gpu_pixels(packed, cam, off, channels, pix):
    """Gather pixels [npix][2] of view at packed offset `off` -> [npix] or [npix][C]."""
    H, W = cam.height, cam.width
    i, j = pix[:, 0], pix[:, 1]
    if channels == 1:
        img = packed[off:off + H * W].reshape(H, W)
        return img[j, i]
    img = packed[3 * off:3 * off + 3 * H * W].reshape(3, H, W)
    return img[:, j, i].T


def crops(cam, size, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        x0 = int(rng.integers(0, max(1, cam.width - size)))
        y0 = int(rng.integers(0, max(1, cam.height - size)))
        out.append((x0, y0, min(size, cam.width - x0), min(size, cam.height - y0)))
    return out


def box_pixels(O, boxes):
    """The pixels [npix][2] (i, j) covered by a list of crop boxes, each once (boxes may
    overlap, and a pixel listed twice would count twice in the oracle's sums)."""
    pix = np.concatenate([O.crop_pixels(*b) for b in boxes])
    pix = np.unique(pix[:, [1, 0]], axis=0)[:, [1, 0]]
    return np.ascontiguousarray(pix, dtype=np.int32)


def crop_mask(cam, boxes):
    m = np.zeros((cam.height, cam.width), dtype=bool)
    for (x0, y0, w, h) in boxes:
        m[y0:y0 + h, x0:x0 + w] = True
    return m


def frame_layout(n_tiles, n_pixels, n_records):
    """Byte offsets inside a frame state (internal layout of libgspm, for tests only)."""
    a = lambda x: (x + 255) & ~255  # noqa: E731
    o = 0
    lay = {}
    lay["header"] = o; o += a(64)
    lay["visible"] = o; o += a(n_records)
    lay["ranges"] = o; o += a(n_tiles * 8)
    lay["t_final"] = o; o += a(n_pixels * 4)
    lay["last"] = o; o += a(n_pixels * 4)
    lay["contrib"] = o; o += a(n_pixels * 4)
    lay["order"] = o; o += a(2 * n_tiles * 4)
    lay["records"] = o; o += a(n_records * 64)
    lay["pair_vals"] = o
    return lay


def tile_edge_near(bounds, B, W, H, tol):
    """True where a support bound is within tol of a value at which the tile rectangle
    (or the visibility) changes: u - rx at k B - 1 (ceil crosses into tile k), u + rx at
    k B (floor crosses), and the image borders."""
    lo_x, hi_x, lo_y, hi_y = bounds[:, 0], bounds[:, 1], bounds[:, 2], bounds[:, 3]
    tol = np.broadcast_to(np.asarray(tol, dtype=np.float64), lo_x.shape)

    def near(x, offs, extra):
        r = np.zeros(x.shape, dtype=bool)
        k = np.round((x - offs) / B)
        r |= np.abs(x - (k * B + offs)) <= tol
        for e in extra:
            r |= np.abs(x - e) <= tol
        return r

    return (near(lo_x, -1.0, [0.0, W - 1.0, W]) | near(hi_x, 0.0, [-1.0, 0.0, W - 1.0]) |
            near(lo_y, -1.0, [0.0, H - 1.0, H]) | near(hi_y, 0.0, [-1.0, 0.0, H - 1.0]))
