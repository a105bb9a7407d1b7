"""ctypes binding of libgspm.so, the C ABI declared in ``include/gspm.h``.

Argument marshalling only: every function here forwards device pointers (taken from
torch tensors) and sizes to the HIP library and raises ``GspmError`` on a non-OK
status.  Nothing is computed in Python and there is no fallback: if the library is
missing the first call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgspm.so")

GSPM_OK, GSPM_ERR_INVALID_ARG, GSPM_ERR_CAPACITY, GSPM_ERR_HIP, GSPM_ERR_INTERNAL = 0, 1, 2, 3, 4
MAX_VIEWS = 32

vp = ctypes.c_void_p
fp = ctypes.POINTER(ctypes.c_float)


class GspmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"gspm status {status}: {message}")
        self.status = status


class CapacityError(GspmError):
    def __init__(self, status, message, pairs):
        super().__init__(status, message)
        self.pairs = pairs


class Gaussians(ctypes.Structure):
    _fields_ = [("means", vp), ("log_scales", vp), ("quats", vp), ("opacity_logit", vp), ("rgb", vp),
                ("n", ctypes.c_int64)]


class Intrinsics(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float)]


class Views(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("intr", ctypes.POINTER(Intrinsics)), ("T_cw", vp)]


class Settings(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("sort_digit_bits", ctypes.c_int32), ("pointmap_frame", ctypes.c_int32),
                ("pixels_per_lane", ctypes.c_int32), ("near_z", ctypes.c_float), ("alpha_min", ctypes.c_float),
                ("alpha_max", ctypes.c_float), ("t_min", ctypes.c_float), ("eps2d", ctypes.c_float),
                ("jac_clamp", ctypes.c_float), ("bg", ctypes.c_float * 3), ("mark_visible", ctypes.c_int32),
                ("count_work", ctypes.c_int32), ("bwd_lane_reduce", ctypes.c_int32),
                ("grads_overwrite", ctypes.c_int32)]


class Images(ctypes.Structure):
    _fields_ = [("rgb", vp), ("depth", vp), ("alpha", vp), ("pointmap", vp)]


class GaussianGrads(ctypes.Structure):
    _fields_ = [("means", vp), ("log_scales", vp), ("quats", vp), ("opacity_logit", vp), ("rgb", vp)]


class PnpParams(ctypes.Structure):
    _fields_ = [("n_hypotheses", ctypes.c_int32), ("threshold", ctypes.c_float), ("iterations", ctypes.c_int32),
                ("rounds", ctypes.c_int32)]


class AlignParams(ctypes.Structure):
    _fields_ = [("patch", ctypes.c_int32), ("delta_mu", ctypes.c_float), ("delta_sigma", ctypes.c_float),
                ("eps_r", ctypes.c_float), ("max_iter", ctypes.c_int32), ("tau", ctypes.c_float)]


# gspm_align_result as stored in device memory (24 bytes per view).
ALIGN_RESULT_DTYPE = np.dtype([("scale", "<f8"), ("cp", "<i4"), ("n_valid", "<i4"), ("insufficient", "<i4"),
                               ("pad", "<i4")])


@dataclass
class AlignConfig:
    """Parameters of the patch-based scale alignment (the paper's values by default)."""
    patch: int = 10
    delta_mu: float = 0.3
    delta_sigma: float = 0.3
    eps_r: float = 0.1
    max_iter: int = 3
    tau: float = 0.01
    eps_m: float = 0.15  # pointmap replacement threshold (Eq. 14)

    def c(self) -> AlignParams:
        return AlignParams(self.patch, self.delta_mu, self.delta_sigma, self.eps_r, self.max_iter, self.tau)


EXPORTS = (
    "gspm_create", "gspm_destroy", "gspm_reserve", "gspm_frame_state_bytes", "gspm_render_forward",
    "gspm_frame_status", "gspm_render_backward", "gspm_pose_backward", "gspm_patch_scale_align",
    "gspm_window_loss", "gspm_pose_retract", "gspm_timing_enable", "gspm_timing_collect", "gspm_frame_work",
    "gspm_last_error", "gspm_version", "gspm_align_scale", "gspm_replace_pointmap", "gspm_iso_loss",
    "gspm_covisibility", "gspm_median_depth", "gspm_pnp_ransac", "gspm_window_loss_noalloc",
)

PHASES = ("preprocess", "depth_sort", "binning", "tile_sort", "raster_fwd", "raster_bwd", "param_bwd")

_lib = None


def load(path: str = LIB_PATH):
    """Open libgspm.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise GspmError(-1, f"{path} not found: build it with `python -m paper_2507_03737_amd.build`")
    L = ctypes.CDLL(path)
    P = ctypes.POINTER
    L.gspm_create.argtypes = [P(vp)]
    L.gspm_destroy.argtypes = [vp]
    L.gspm_destroy.restype = None
    L.gspm_reserve.argtypes = [vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
    L.gspm_frame_state_bytes.argtypes = [P(Views), ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
    L.gspm_frame_state_bytes.restype = ctypes.c_int64
    L.gspm_render_forward.argtypes = [vp, P(Gaussians), P(Views), P(Settings), P(Images), vp, ctypes.c_int64, vp]
    L.gspm_frame_status.argtypes = [vp, vp, P(ctypes.c_int64)]
    L.gspm_render_backward.argtypes = [vp, P(Gaussians), P(Views), P(Settings), P(Images), P(Images), vp,
                                       P(GaussianGrads), vp, vp]
    L.gspm_pose_backward.argtypes = [vp, P(Gaussians), P(Views), P(Settings), P(Images), P(Images), vp, vp, vp]
    L.gspm_patch_scale_align.argtypes = [P(Views), vp, vp, vp, ctypes.c_int32, vp, vp, vp]
    L.gspm_window_loss.argtypes = [vp, P(Views), vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float, vp, vp, vp, vp, vp]
    L.gspm_window_loss_noalloc.argtypes = [P(Views), vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float, vp, vp, vp,
                                           vp, vp]
    L.gspm_pose_retract.argtypes = [ctypes.c_int32, vp, vp, vp]
    L.gspm_align_scale.argtypes = [vp, P(Views), vp, vp, vp, P(AlignParams), vp, vp]
    L.gspm_replace_pointmap.argtypes = [P(Views), vp, vp, vp, ctypes.c_float, vp, vp, vp]
    L.gspm_iso_loss.argtypes = [vp, P(Gaussians), ctypes.c_float, vp, vp, vp]
    L.gspm_covisibility.argtypes = [vp, P(Views), ctypes.c_int64, vp, vp, vp, vp, vp]
    L.gspm_median_depth.argtypes = [vp, P(Views), vp, vp, vp]
    L.gspm_pnp_ransac.argtypes = [vp, vp, vp, ctypes.c_int64, P(Intrinsics), vp, P(PnpParams), vp, vp, vp, vp, vp,
                                  vp, vp]
    L.gspm_frame_work.argtypes = [vp, P(Views), ctypes.c_int64, ctypes.c_int32, vp, vp, P(ctypes.c_int64)]
    L.gspm_timing_enable.argtypes = [vp, ctypes.c_int32]
    L.gspm_timing_collect.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.gspm_last_error.restype = ctypes.c_char_p
    L.gspm_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        getattr(L, name)
    _lib = L
    return L


def last_error() -> str:
    return load().gspm_last_error().decode()


def check(status: int):
    if status != GSPM_OK:
        raise GspmError(status, last_error())


def ptr(t) -> int | None:
    """Device pointer of a tensor (None for None)."""
    return None if t is None else t.data_ptr()


def stream_handle(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


@dataclass
class RasterConfig:
    """Settings of the rasterizer (see gspm_settings)."""
    tile: int = 16
    sort_digit_bits: int = 8
    pointmap_frame: int = 1
    pixels_per_lane: int = 1
    near_z: float = 0.2
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    eps2d: float = 0.3
    jac_clamp: float = 1.3
    bg: tuple = (0.0, 0.0, 0.0)
    mark_visible: int = 0
    count_work: int = 0
    bwd_lane_reduce: int = 0
    grads_overwrite: int = 0

    def c(self) -> Settings:
        return Settings(self.tile, self.sort_digit_bits, self.pointmap_frame, self.pixels_per_lane, self.near_z,
                        self.alpha_min,
                        self.alpha_max, self.t_min, self.eps2d, self.jac_clamp, (ctypes.c_float * 3)(*self.bg),
                        int(self.mark_visible), int(self.count_work), int(self.bwd_lane_reduce),
                        int(self.grads_overwrite))

    # Supported (tile, pixels_per_lane) launch shapes of the raster kernels.
    SHAPES = ((8, 1), (16, 1), (16, 2), (16, 4), (32, 1), (32, 2), (32, 4))

    def with_shape(self, tile, ppl):
        import dataclasses
        return dataclasses.replace(self, tile=tile, pixels_per_lane=ppl)


def make_intrinsics(cams):
    arr = (Intrinsics * len(cams))()
    for k, c in enumerate(cams):
        arr[k] = Intrinsics(int(c.width), int(c.height), float(c.fx), float(c.fy), float(c.cx), float(c.cy))
    return arr


def make_views(intr_arr, n_views, T_cw) -> Views:
    return Views(n_views, ctypes.cast(intr_arr, ctypes.POINTER(Intrinsics)), ptr(T_cw))


def make_gaussians(means, log_scales, quats, opacity_logit, rgb) -> Gaussians:
    return Gaussians(ptr(means), ptr(log_scales), ptr(quats), ptr(opacity_logit), ptr(rgb), int(means.shape[-1]))


class Context:
    """Owns a gspm_ctx (scratch memory for sorts and per-record gradients)."""

    def __init__(self):
        L = load()
        h = vp()
        check(L.gspm_create(ctypes.byref(h)))
        self.h = h

    def reserve(self, max_records, max_pairs, max_tiles=0):
        check(load().gspm_reserve(self.h, int(max_records), int(max_pairs), int(max_tiles)))

    def timing(self, on: bool):
        check(load().gspm_timing_enable(self.h, 1 if on else 0))

    def collect_timing(self):
        """Per-phase (total ms, launches) since the last collect; synchronises."""
        ms = (ctypes.c_double * len(PHASES))()
        cnt = (ctypes.c_int64 * len(PHASES))()
        check(load().gspm_timing_collect(self.h, ms, cnt))
        return {p: (ms[k], int(cnt[k])) for k, p in enumerate(PHASES)}

    def close(self):
        if self.h:
            load().gspm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def frame_state_bytes(views: Views, n, max_pairs, tile) -> int:
    b = load().gspm_frame_state_bytes(ctypes.byref(views), int(n), int(max_pairs), int(tile))
    if b < 0:
        raise GspmError(GSPM_ERR_INVALID_ARG, last_error())
    return int(b)


def render_forward(ctx: Context, g: Gaussians, views: Views, cfg: Settings, out: Images, frame_state, stream):
    check(load().gspm_render_forward(ctx.h, ctypes.byref(g), ctypes.byref(views), ctypes.byref(cfg),
                                     ctypes.byref(out), ptr(frame_state), frame_state.numel(), stream))


def frame_status(frame_state, stream) -> int:
    pairs = ctypes.c_int64(0)
    st = load().gspm_frame_status(ptr(frame_state), stream, ctypes.byref(pairs))
    if st == GSPM_ERR_CAPACITY:
        raise CapacityError(st, last_error(), int(pairs.value))
    check(st)
    return int(pairs.value)


def frame_work(ctx: Context, views: Views, n, tile, frame_state, stream):
    """(tile pairs, contributing fragments, evaluated-list bound, walked wave entries,
    accepted wave entries) of a counting forward; synchronises."""
    out = (ctypes.c_int64 * 5)()
    check(load().gspm_frame_work(ctx.h, ctypes.byref(views), int(n), int(tile), ptr(frame_state), stream, out))
    return tuple(int(x) for x in out)


def render_backward(ctx, g, views, cfg, fwd: Images, up: Images, frame_state, grads: GaussianGrads | None,
                    pose_grad, stream):
    check(load().gspm_render_backward(ctx.h, ctypes.byref(g), ctypes.byref(views), ctypes.byref(cfg),
                                      ctypes.byref(fwd), ctypes.byref(up), ptr(frame_state),
                                      ctypes.byref(grads) if grads is not None else None, ptr(pose_grad), stream))


def pose_backward(ctx, g, views, cfg, fwd: Images, up: Images, frame_state, pose_grad, stream):
    check(load().gspm_pose_backward(ctx.h, ctypes.byref(g), ctypes.byref(views), ctypes.byref(cfg),
                                    ctypes.byref(fwd), ctypes.byref(up), ptr(frame_state), ptr(pose_grad), stream))


def patch_scale_align(views: Views, Xr, Xp, mask, patch, scale_out, count_out, stream):
    check(load().gspm_patch_scale_align(ctypes.byref(views), ptr(Xr), ptr(Xp), ptr(mask), int(patch),
                                        ptr(scale_out), ptr(count_out), stream))


def window_loss(ctx: Context, views: Views, rgb, rgb_target, pm, Xp, patch, alpha, scale_out, loss_out, grad_rgb,
                grad_pm, stream):
    check(load().gspm_window_loss(ctx.h, ctypes.byref(views), ptr(rgb), ptr(rgb_target), ptr(pm), ptr(Xp), int(patch),
                                  float(alpha), ptr(scale_out), ptr(loss_out), ptr(grad_rgb), ptr(grad_pm), stream))


def window_loss_noalloc(views: Views, rgb, rgb_target, pm, Xp, patch, alpha, scale_out, loss_out, grad_rgb, grad_pm,
                        stream):
    """gspm_window_loss without a context: its partial sums use the library's static device array."""
    check(load().gspm_window_loss_noalloc(ctypes.byref(views), ptr(rgb), ptr(rgb_target), ptr(pm), ptr(Xp),
                                          int(patch), float(alpha), ptr(scale_out), ptr(loss_out), ptr(grad_rgb),
                                          ptr(grad_pm), stream))


def align_scale(ctx: Context, views: Views, Xr, Xp, mask, params: AlignParams, result, stream):
    """result: device buffer of 24 * n_views bytes (gspm_align_result per view)."""
    check(load().gspm_align_scale(ctx.h, ctypes.byref(views), ptr(Xr), ptr(Xp), ptr(mask), ctypes.byref(params),
                                  ptr(result), stream))


def replace_pointmap(views: Views, Xr, Xp, result, eps_m, Xr_hat, replaced_out, stream):
    check(load().gspm_replace_pointmap(ctypes.byref(views), ptr(Xr), ptr(Xp), ptr(result), float(eps_m), ptr(Xr_hat),
                                       ptr(replaced_out), stream))


def iso_loss(ctx: Context, g: Gaussians, weight, loss_out, grad_log_scales, stream):
    check(load().gspm_iso_loss(ctx.h, ctypes.byref(g), float(weight), ptr(loss_out), ptr(grad_log_scales), stream))


def covisibility(ctx: Context, views: Views, n, frame_state, iou_out, oc_out, count_out, stream):
    check(load().gspm_covisibility(ctx.h, ctypes.byref(views), int(n), ptr(frame_state), ptr(iou_out), ptr(oc_out),
                                   ptr(count_out), stream))


def median_depth(ctx: Context, views: Views, depth, median_out, stream):
    check(load().gspm_median_depth(ctx.h, ctypes.byref(views), ptr(depth), ptr(median_out), stream))


def pnp_ransac(ctx: Context, X, uv, K: Intrinsics, samples, params: PnpParams, T_out, n_inliers, mask, scores,
               T_ak, T_n_out, stream):
    check(load().gspm_pnp_ransac(ctx.h, ptr(X), ptr(uv), int(X.shape[-1]), ctypes.byref(K), ptr(samples),
                                 ctypes.byref(params), ptr(T_out), ptr(n_inliers), ptr(mask), ptr(scores),
                                 ptr(T_ak), ptr(T_n_out), stream))


def pose_retract(n_views, T_cw, xi, stream):
    check(load().gspm_pose_retract(int(n_views), ptr(T_cw), ptr(xi), stream))


def version() -> str:
    return load().gspm_version().decode()


def np_intrinsics(cams):
    return np.array([[c.width, c.height, c.fx, c.fy, c.cx, c.cy] for c in cams], dtype=np.float64)
