"""Python front end of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the benchmark's
CPU-baseline leg.  The product path never imports it.

The per-pixel renderer, its analytic backward, the frozen-decision replay used for
finite differences and the tile lists of the supports live in ``gs_oracle.c`` (plain C,
double precision, OpenMP over pixels).  This module marshals arrays for it and adds
the two oracle steps that are short enough to state directly in numpy:

* ``patch_scale``: per-patch least-squares scale between a prior pointmap and the
  rendered one (the per-patch scale fit that aligns the pre-trained pointmap to the
  scene, Sec. 3.3.1; here the least-squares estimator per P x P patch).
* ``l1_window_loss``: the mapping objective of Eq. 17 restricted to its photometric
  (Eq. 10) and pointmap (Eq. 15) terms, alpha L_pho + (1 - alpha) L_geo, with the
  patch scale held constant, and its gradient with respect to the rendered images.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

f64p = ctypes.POINTER(ctypes.c_double)
i32p = ctypes.POINTER(ctypes.c_int32)
i64p = ctypes.POINTER(ctypes.c_int64)
i8p = ctypes.POINTER(ctypes.c_int8)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wno-unused-function", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Gaussians(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("means", f64p), ("log_scales", f64p), ("quats", f64p),
                ("opacity_logit", f64p), ("rgb", f64p)]


class _View(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_double),
                ("fy", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double),
                ("T", ctypes.c_double * 12)]


class _Settings(ctypes.Structure):
    _fields_ = [("near_z", ctypes.c_double), ("alpha_min", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("t_min", ctypes.c_double),
                ("eps2d", ctypes.c_double), ("jac_clamp", ctypes.c_double),
                ("bg", ctypes.c_double * 3), ("flag_factor", ctypes.c_double)]


class _Proj(ctypes.Structure):
    _fields_ = [("visible", ctypes.c_int32), ("clamp_x", ctypes.c_int32), ("clamp_y", ctypes.c_int32),
                ("rect", ctypes.c_int32 * 4), ("cand", ctypes.c_int32), ("crect", ctypes.c_int32 * 4),
                ("m", ctypes.c_double * 3), ("u", ctypes.c_double),
                ("v", ctypes.c_double), ("z", ctypes.c_double), ("a", ctypes.c_double),
                ("s", ctypes.c_double * 3), ("qn", ctypes.c_double * 4), ("qnorm", ctypes.c_double),
                ("Rq", ctypes.c_double * 9), ("Sig", ctypes.c_double * 9), ("Sigc", ctypes.c_double * 9),
                ("J", ctypes.c_double * 6), ("cov2", ctypes.c_double * 3), ("Q", ctypes.c_double * 3),
                ("rx", ctypes.c_double), ("ry", ctypes.c_double), ("bounds", ctypes.c_double * 4)]


class _Pixel(ctypes.Structure):
    _fields_ = [("rgb", ctypes.c_double * 3), ("depth", ctypes.c_double), ("alpha", ctypes.c_double),
                ("pm_world", ctypes.c_double * 3), ("pm_cam", ctypes.c_double * 3),
                ("pm_eq5", ctypes.c_double * 3), ("T_final", ctypes.c_double),
                ("n_frag", ctypes.c_int32), ("n_cand", ctypes.c_int32),
                ("ambiguous", ctypes.c_int32), ("pad", ctypes.c_int32), ("margin", ctypes.c_double)]


class _Grads(ctypes.Structure):
    _fields_ = [("means", f64p), ("log_scales", f64p), ("quats", f64p), ("opacity_logit", f64p),
                ("rgb", f64p), ("pose", f64p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        L.orc_project.argtypes = [ctypes.POINTER(_Gaussians), ctypes.POINTER(_View),
                                  ctypes.POINTER(_Settings), ctypes.POINTER(_Proj)]
        L.orc_render.argtypes = [ctypes.POINTER(_Gaussians), ctypes.POINTER(_View),
                                 ctypes.POINTER(_Settings), ctypes.POINTER(_Proj), ctypes.c_int64,
                                 i32p, ctypes.POINTER(_Pixel)]
        L.orc_trace.argtypes = [ctypes.POINTER(_Gaussians), ctypes.POINTER(_View),
                                ctypes.POINTER(_Settings), ctypes.POINTER(_Proj), ctypes.c_int64,
                                i32p, ctypes.c_int64, i64p, i64p, i8p]
        L.orc_trace.restype = ctypes.c_int64
        L.orc_replay_loss.argtypes = [ctypes.POINTER(_Gaussians), ctypes.POINTER(_View),
                                      ctypes.POINTER(_Settings), i8p, ctypes.c_int32, ctypes.c_int64,
                                      i32p, i64p, i64p, i8p, f64p, f64p, f64p, f64p]
        L.orc_replay_loss.restype = ctypes.c_double
        L.orc_backward.argtypes = [ctypes.POINTER(_Gaussians), ctypes.POINTER(_View),
                                   ctypes.POINTER(_Settings), ctypes.POINTER(_Proj), ctypes.c_int32,
                                   ctypes.c_int64, i32p, f64p, f64p, f64p, f64p,
                                   ctypes.POINTER(_Grads)]
        L.orc_tile_sets.argtypes = [ctypes.POINTER(_Proj), ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_int64, i32p,
                                    i64p, f64p]
        L.orc_tile_sets.restype = ctypes.c_int64
        L.orc_se3_exp_left.argtypes = [f64p, f64p, f64p]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _p(a, t=f64p):
    return a.ctypes.data_as(t)


@dataclass
class Settings:
    """Rasterizer conventions (values as the float32 numbers the library receives)."""
    near_z: float = 0.2
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    eps2d: float = 0.3
    jac_clamp: float = 1.3
    bg: tuple = (0.0, 0.0, 0.0)
    # A pixel is flagged as ambiguous when one of its alpha_min, alpha_max or t_min
    # decisions lies within flag_factor first-order float32 error bounds of its threshold.
    flag_factor: float = 1.0

    def c(self):
        f = lambda x: float(np.float32(x))  # noqa: E731
        return _Settings(f(self.near_z), f(self.alpha_min), f(self.alpha_max), f(self.t_min),
                         f(self.eps2d), f(self.jac_clamp), (ctypes.c_double * 3)(*[f(b) for b in self.bg]),
                         float(self.flag_factor))


class Params:
    """Float64 copies of a Gaussian set (planar SoA), kept alive for ctypes."""

    def __init__(self, means, log_scales, quats, opacity_logit, rgb):
        self.means = np.ascontiguousarray(means, dtype=np.float64)
        self.log_scales = np.ascontiguousarray(log_scales, dtype=np.float64)
        self.quats = np.ascontiguousarray(quats, dtype=np.float64)
        self.opacity_logit = np.ascontiguousarray(opacity_logit, dtype=np.float64)
        self.rgb = np.ascontiguousarray(rgb, dtype=np.float64)
        self.n = self.means.shape[1]
        self._c = _Gaussians(self.n, _p(self.means), _p(self.log_scales), _p(self.quats),
                             _p(self.opacity_logit), _p(self.rgb))

    @staticmethod
    def from_scene(scene):
        return Params(*scene.params())

    def copy(self):
        return Params(self.means.copy(), self.log_scales.copy(), self.quats.copy(),
                      self.opacity_logit.copy(), self.rgb.copy())

    def flat(self):
        return [self.means, self.log_scales, self.quats, self.opacity_logit, self.rgb]


def make_view(cam, T12):
    T = np.asarray(T12, dtype=np.float64).reshape(12)
    return _View(int(cam.width), int(cam.height), float(np.float32(cam.fx)), float(np.float32(cam.fy)),
                 float(np.float32(cam.cx)), float(np.float32(cam.cy)), (ctypes.c_double * 12)(*T))


def full_pixels(cam):
    jj, ii = np.meshgrid(np.arange(cam.height, dtype=np.int32), np.arange(cam.width, dtype=np.int32),
                         indexing="ij")
    return np.ascontiguousarray(np.stack([ii.reshape(-1), jj.reshape(-1)], axis=1))


def crop_pixels(x0, y0, w, h):
    jj, ii = np.meshgrid(np.arange(y0, y0 + h, dtype=np.int32), np.arange(x0, x0 + w, dtype=np.int32),
                         indexing="ij")
    return np.ascontiguousarray(np.stack([ii.reshape(-1), jj.reshape(-1)], axis=1))


def project(params: Params, view, settings: Settings):
    """Per-Gaussian projection records (numpy structured array of length n)."""
    arr = (_Proj * params.n)()
    lib().orc_project(ctypes.byref(params._c), ctypes.byref(view), ctypes.byref(settings.c()), arr)
    return arr


def proj_numpy(arr):
    return np.ctypeslib.as_array(arr)


def render(params: Params, view, settings: Settings, pixels, proj=None):
    """Render the given pixels ([npix][2] int32 (i, j)).  Returns a dict of float64 arrays."""
    proj = project(params, view, settings) if proj is None else proj
    pixels = np.ascontiguousarray(pixels, dtype=np.int32)
    npix = pixels.shape[0]
    out = (_Pixel * npix)()
    rc = lib().orc_render(ctypes.byref(params._c), ctypes.byref(view), ctypes.byref(settings.c()),
                          proj, npix, _p(pixels, i32p), out)
    if rc != 0:
        raise MemoryError("oracle render failed")
    a = np.ctypeslib.as_array(out)
    return {
        "rgb": np.array(a["rgb"]), "depth": np.array(a["depth"]), "alpha": np.array(a["alpha"]),
        "pm_world": np.array(a["pm_world"]), "pm_cam": np.array(a["pm_cam"]),
        "pm_eq5": np.array(a["pm_eq5"]), "T_final": np.array(a["T_final"]),
        "n_frag": np.array(a["n_frag"]), "n_cand": np.array(a["n_cand"]),
        "ambiguous": np.array(a["ambiguous"]), "margin": np.array(a["margin"]),
    }


def render_image(params: Params, cam, T12, settings: Settings):
    """Full-frame render reshaped to planar images ([3][H][W], [H][W], ...)."""
    view = make_view(cam, T12)
    pix = full_pixels(cam)
    r = render(params, view, settings, pix)
    H, W = cam.height, cam.width
    img = {}
    for k in ("rgb", "pm_world", "pm_cam", "pm_eq5"):
        img[k] = r[k].reshape(H, W, 3).transpose(2, 0, 1).copy()
    for k in ("depth", "alpha", "T_final", "n_frag", "n_cand", "ambiguous", "margin"):
        img[k] = r[k].reshape(H, W)
    return img


class Trace:
    def __init__(self, offsets, frag_g, frag_clamped, clamp_xy, pixels):
        self.offsets, self.frag_g, self.frag_clamped = offsets, frag_g, frag_clamped
        self.clamp_xy, self.pixels = clamp_xy, pixels


def trace(params: Params, view, settings: Settings, pixels):
    proj = project(params, view, settings)
    pixels = np.ascontiguousarray(pixels, dtype=np.int32)
    npix = pixels.shape[0]
    offsets = np.zeros(npix + 1, dtype=np.int64)
    cap = 0
    dummy_g = np.zeros(1, dtype=np.int64)
    dummy_c = np.zeros(1, dtype=np.int8)
    L = lib()
    need = L.orc_trace(ctypes.byref(params._c), ctypes.byref(view), ctypes.byref(settings.c()), proj,
                       npix, _p(pixels, i32p), cap, _p(offsets, i64p), _p(dummy_g, i64p),
                       _p(dummy_c, i8p))
    total = -need if need < 0 else need
    frag_g = np.zeros(max(total, 1), dtype=np.int64)
    frag_c = np.zeros(max(total, 1), dtype=np.int8)
    got = L.orc_trace(ctypes.byref(params._c), ctypes.byref(view), ctypes.byref(settings.c()), proj,
                      npix, _p(pixels, i32p), total, _p(offsets, i64p), _p(frag_g, i64p),
                      _p(frag_c, i8p))
    assert got == total
    pa = proj_numpy(proj)
    clamp = np.ascontiguousarray(np.stack([pa["clamp_x"], pa["clamp_y"]], axis=1).astype(np.int8))
    return Trace(offsets, frag_g, frag_c, clamp, pixels)


def replay_loss(params: Params, view, settings: Settings, tr: Trace, up, pointmap_frame=0):
    """L = sum over traced pixels of g . outputs, with the trace's discrete decisions frozen.

    ``up`` holds per-pixel upstream gradients: rgb [npix][3], depth [npix], alpha [npix],
    pointmap [npix][3] (float64)."""
    return lib().orc_replay_loss(
        ctypes.byref(params._c), ctypes.byref(view), ctypes.byref(settings.c()),
        _p(tr.clamp_xy, i8p), int(pointmap_frame), tr.pixels.shape[0], _p(tr.pixels, i32p),
        _p(tr.offsets, i64p), _p(tr.frag_g, i64p), _p(tr.frag_clamped, i8p),
        _p(up["rgb"]), _p(up["depth"]), _p(up["alpha"]), _p(up["pointmap"]))


def pixel_upstream(up_img, pixels):
    """Gather planar upstream images at pixels -> per-pixel float64 arrays."""
    i, j = pixels[:, 0], pixels[:, 1]
    return {
        "rgb": np.ascontiguousarray(up_img["rgb"][:, j, i].T, dtype=np.float64),
        "depth": np.ascontiguousarray(up_img["depth"][j, i], dtype=np.float64),
        "alpha": np.ascontiguousarray(up_img["alpha"][j, i], dtype=np.float64),
        "pointmap": np.ascontiguousarray(up_img["pointmap"][:, j, i].T, dtype=np.float64),
    }


def backward(params: Params, view, settings: Settings, pixels, up, pointmap_frame=0, proj=None):
    """Analytic VJP for the given pixels and per-pixel upstream gradients.

    Returns dict of float64 gradients: means [3][n], log_scales [3][n], quats [4][n],
    opacity_logit [n], rgb [3][n], pose [6] (left se(3) perturbation, rho first)."""
    proj = project(params, view, settings) if proj is None else proj
    n = params.n
    g = {"means": np.zeros((3, n)), "log_scales": np.zeros((3, n)), "quats": np.zeros((4, n)),
         "opacity_logit": np.zeros(n), "rgb": np.zeros((3, n)), "pose": np.zeros(6)}
    cg = _Grads(_p(g["means"]), _p(g["log_scales"]), _p(g["quats"]), _p(g["opacity_logit"]),
                _p(g["rgb"]), _p(g["pose"]))
    pixels = np.ascontiguousarray(pixels, dtype=np.int32)
    rc = lib().orc_backward(ctypes.byref(params._c), ctypes.byref(view), ctypes.byref(settings.c()),
                            proj, int(pointmap_frame), pixels.shape[0], _p(pixels, i32p),
                            _p(up["rgb"]), _p(up["depth"]), _p(up["alpha"]), _p(up["pointmap"]),
                            ctypes.byref(cg))
    if rc != 0:
        raise MemoryError("oracle backward failed")
    return g


def tile_sets(proj, n, width, height, B, settings=None):
    """Tile lists of the supports for tile size B (the tile-based rasterization of
    Sec. 3.1), ordered by (tile, z, index).  Returns (tiles, gaussians, ratio) for the
    *rect* pairs (the tile holds a pixel of the Gaussian's support box); the pair is also
    in the *exact* set (the tile holds a pixel centre where the Gaussian's alpha reaches
    alpha_min) iff ratio <= 1, ratio being the smallest Mahalanobis term over the tile's
    pixels of the box divided by the support level 2 ln(a / alpha_min)."""
    s = settings or Settings()
    amin = float(np.float32(s.alpha_min))
    L = lib()
    need = L.orc_tile_sets(proj, n, width, height, B, amin, 0, None, None, None)
    total = -need if need < 0 else need
    tiles = np.zeros(max(total, 1), dtype=np.int32)
    gs = np.zeros(max(total, 1), dtype=np.int64)
    ratio = np.zeros(max(total, 1), dtype=np.float64)
    got = L.orc_tile_sets(proj, n, width, height, B, amin, total, _p(tiles, i32p), _p(gs, i64p), _p(ratio))
    assert got == total
    return tiles[:total], gs[:total], ratio[:total]


def se3_exp_left(xi, T12):
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    T = np.ascontiguousarray(np.asarray(T12, dtype=np.float64).reshape(12))
    out = np.zeros(12)
    lib().orc_se3_exp_left(_p(xi), _p(T), _p(out))
    return out


def num_threads():
    return int(lib().orc_num_threads())


def set_num_threads(n: int):
    """Threads the oracle's parallel loops use from now on (OpenMP)."""
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# Patch least-squares scale and the window loss (numpy).

def patch_scale(Xr, Xp, P, mask=None):
    """Per-patch least-squares scale s minimising sum |Xr - s Xp|^2 over each P x P patch.

    Xr, Xp: [3][H][W]; mask: [H][W] (nonzero = use) or None.  Border patches are partial.
    Returns (scale [ceil(H/P)][ceil(W/P)], count [same]); a patch whose sum |Xp|^2 is
    zero gets scale 1 (count is then the number of masked pixels, which may be 0)."""
    Xr = np.asarray(Xr, dtype=np.float64)
    Xp = np.asarray(Xp, dtype=np.float64)
    _, H, W = Xr.shape
    m = np.ones((H, W)) if mask is None else (np.asarray(mask) != 0).astype(np.float64)
    nph, npw = -(-H // P), -(-W // P)
    scale = np.ones((nph, npw))
    count = np.zeros((nph, npw), dtype=np.int64)
    sxy_img = (Xr * Xp).sum(axis=0) * m
    syy_img = (Xp * Xp).sum(axis=0) * m
    for py in range(nph):
        for px in range(npw):
            sl = (slice(py * P, min(H, (py + 1) * P)), slice(px * P, min(W, (px + 1) * P)))
            sxy = sxy_img[sl].sum()
            syy = syy_img[sl].sum()
            count[py, px] = int(m[sl].sum())
            if syy > 0.0:
                scale[py, px] = sxy / syy
    return scale, count


def expand_patches(scale, P, H, W):
    """Per-pixel view of a per-patch array."""
    return np.repeat(np.repeat(scale, P, axis=0), P, axis=1)[:H, :W]


def l1_window_loss(rgb, rgb_target, pm, prior, scale, P, alpha=0.98):
    """alpha * mean|rgb - target| + (1 - alpha) * mean|pm - s * prior| for one view.

    The per-patch scale s is a constant (no gradient flows into it).  Returns
    (loss, d loss / d rgb, d loss / d pm); the sign of 0 is 0."""
    rgb = np.asarray(rgb, dtype=np.float64)
    pm = np.asarray(pm, dtype=np.float64)
    _, H, W = rgb.shape
    s = expand_patches(np.asarray(scale, dtype=np.float64), P, H, W)
    r_pho = rgb - np.asarray(rgb_target, dtype=np.float64)
    r_geo = pm - s[None] * np.asarray(prior, dtype=np.float64)
    n_pho = r_pho.size
    n_geo = r_geo.size
    loss = alpha * np.abs(r_pho).sum() / n_pho + (1.0 - alpha) * np.abs(r_geo).sum() / n_geo
    return loss, alpha * np.sign(r_pho) / n_pho, (1.0 - alpha) * np.sign(r_geo) / n_geo
