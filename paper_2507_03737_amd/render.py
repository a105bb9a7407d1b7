"""Python layer over the C ABI: packed view windows, capacity handling, the autograd
function and the graph-captured mapping iteration.

Tensors are only allocated and passed by pointer here; every step of rendering, the
backward, the patch scale and the loss runs in libgspm's HIP kernels.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import torch

from . import binding as B

__all__ = ["Window", "Rasterizer", "RasterizePointmap", "rasterize", "MappingStep", "AutogradMappingStep",
           "split_views", "align_results"]


class Window:
    """A window of views (keyframes): host intrinsics and device poses T_cw [V][12]."""

    def __init__(self, cams: Sequence, T_cw: torch.Tensor):
        if len(cams) < 1 or len(cams) > B.MAX_VIEWS:
            raise ValueError(f"need 1..{B.MAX_VIEWS} views")
        if T_cw.dtype != torch.float32 or not T_cw.is_cuda or tuple(T_cw.shape) != (len(cams), 12):
            raise ValueError("T_cw must be a float32 CUDA tensor of shape [V, 12]")
        self.cams = list(cams)
        self.T_cw = T_cw.contiguous()
        self._intr = B.make_intrinsics(self.cams)
        self.sizes = [(int(c.height), int(c.width)) for c in self.cams]
        self.pix_off = [0]
        for h, w in self.sizes:
            self.pix_off.append(self.pix_off[-1] + h * w)
        self.n_pixels = self.pix_off[-1]

    @property
    def n_views(self):
        return len(self.cams)

    def c(self) -> B.Views:
        return B.make_views(self._intr, self.n_views, self.T_cw)

    def n_tiles(self, tile):
        return sum(math.ceil(w / tile) * math.ceil(h / tile) for h, w in self.sizes)

    def n_patches(self, patch):
        return sum(math.ceil(w / patch) * math.ceil(h / patch) for h, w in self.sizes)

    def subwindow(self, v: int) -> "Window":
        return Window([self.cams[v]], self.T_cw[v:v + 1])


def split_views(win: Window, packed: torch.Tensor, channels: int) -> List[torch.Tensor]:
    """Views of a packed image buffer as per-view [C][H][W] (or [H][W]) tensors."""
    out = []
    for v, (h, w) in enumerate(win.sizes):
        seg = packed[channels * win.pix_off[v]:channels * win.pix_off[v + 1]]
        out.append(seg.view(channels, h, w) if channels > 1 else seg.view(h, w))
    return out


def _params(params):
    means, log_scales, quats, opacity_logit, rgb = params
    for t, rows in ((means, 3), (log_scales, 3), (quats, 4), (rgb, 3)):
        if t.dtype != torch.float32 or not t.is_cuda or t.dim() != 2 or t.shape[0] != rows or not t.is_contiguous():
            raise ValueError("Gaussian parameters must be contiguous float32 CUDA tensors [rows][n]")
    if opacity_logit.dtype != torch.float32 or opacity_logit.dim() != 1 or not opacity_logit.is_contiguous():
        raise ValueError("opacity_logit must be a contiguous float32 CUDA tensor [n]")
    return B.make_gaussians(means, log_scales, quats, opacity_logit, rgb)


class Rasterizer:
    """Renders a window through libgspm and keeps the scratch context and capacity."""

    def __init__(self, win: Window, n_gaussians: int, cfg: B.RasterConfig | None = None,
                 max_pairs: int | None = None):
        self.win = win
        self.cfg = cfg or B.RasterConfig()
        self.n = int(n_gaussians)
        self.ctx = B.Context()
        # Initial pair capacity: a generous multiple of the pixel count; grown on overflow.
        self.max_pairs = int(max_pairs) if max_pairs else max(1 << 16, 8 * win.n_pixels)
        self.pairs = None
        self.last_frame = None  # frame state of the last forward made through the autograd function

    # -- buffers -----------------------------------------------------------------------
    def frame_bytes(self):
        return B.frame_state_bytes(self.win.c(), self.n, self.max_pairs, self.cfg.tile)

    def new_frame_state(self):
        return torch.empty(self.frame_bytes(), dtype=torch.uint8, device=self.win.T_cw.device)

    def new_outputs(self):
        P = self.win.n_pixels
        dev = self.win.T_cw.device
        return {"rgb": torch.empty(3 * P, device=dev), "depth": torch.empty(P, device=dev),
                "alpha": torch.empty(P, device=dev), "pointmap": torch.empty(3 * P, device=dev)}

    def reserve(self):
        self.ctx.reserve(self.n * self.win.n_views, self.max_pairs, self.win.n_tiles(self.cfg.tile))

    # -- calls -------------------------------------------------------------------------
    def forward_into(self, params, out, frame_state, stream=None):
        g = _params(params)
        img = B.Images(B.ptr(out["rgb"]), B.ptr(out["depth"]), B.ptr(out["alpha"]), B.ptr(out["pointmap"]))
        B.render_forward(self.ctx, g, self.win.c(), self.cfg.c(), img, frame_state, B.stream_handle(stream))

    def forward(self, params, check=True):
        """Render; with check=True, synchronise and grow the pair capacity on overflow."""
        while True:
            out = self.new_outputs()
            fs = self.new_frame_state()
            self.forward_into(params, out, fs)
            if not check:
                return out, fs
            try:
                self.pairs = B.frame_status(fs, B.stream_handle())
                return out, fs
            except B.CapacityError as e:
                self.max_pairs = int(e.pairs * 1.25) + 1024

    def check(self, frame_state=None):
        """Synchronise and read the status of a forward (by default the last one made through
        the autograd function).  On overflow the pair capacity grows and CapacityError is
        raised: that forward's images are incomplete and its backward computed nothing, so
        the step is to be run again (or re-captured)."""
        fs = self.last_frame if frame_state is None else frame_state
        if fs is None:
            raise RuntimeError("no forward to check")
        try:
            self.pairs = B.frame_status(fs, B.stream_handle())
        except B.CapacityError as e:
            self.max_pairs = int(e.pairs * 1.25) + 1024
            raise
        return self.pairs

    def work(self, frame_state, stream=None):
        """(tile pairs, contributing fragments F, evaluated-list bound, walked (wave, entry)
        pairs, accepted (wave, entry) pairs) of a counting forward."""
        return B.frame_work(self.ctx, self.win.c(), self.n, self.cfg.tile, frame_state, B.stream_handle(stream))

    def backward_into(self, params, fwd, up, frame_state, grads=None, pose_grad=None, stream=None,
                      overwrite=False):
        """Backward of a forward into grads / pose_grad: added to their contents, or with
        overwrite=True written over them (no clearing needed)."""
        g = _params(params)
        f = B.Images(B.ptr(fwd["rgb"]), B.ptr(fwd["depth"]), B.ptr(fwd["alpha"]), B.ptr(fwd["pointmap"]))
        u = B.Images(B.ptr(up.get("rgb")), B.ptr(up.get("depth")), B.ptr(up.get("alpha")), B.ptr(up.get("pointmap")))
        gg = None
        if grads is not None:
            gg = B.GaussianGrads(B.ptr(grads.get("means")), B.ptr(grads.get("log_scales")), B.ptr(grads.get("quats")),
                                 B.ptr(grads.get("opacity_logit")), B.ptr(grads.get("rgb")))
        cfg = dataclasses.replace(self.cfg, grads_overwrite=1) if overwrite else self.cfg
        B.render_backward(self.ctx, g, self.win.c(), cfg.c(), f, u, frame_state, gg, pose_grad,
                          B.stream_handle(stream))

    def pose_backward_into(self, params, fwd, up, frame_state, pose_grad, stream=None):
        g = _params(params)
        f = B.Images(B.ptr(fwd["rgb"]), B.ptr(fwd["depth"]), B.ptr(fwd["alpha"]), B.ptr(fwd["pointmap"]))
        u = B.Images(B.ptr(up.get("rgb")), B.ptr(up.get("depth")), B.ptr(up.get("alpha")), B.ptr(up.get("pointmap")))
        B.pose_backward(self.ctx, g, self.win.c(), self.cfg.c(), f, u, frame_state, pose_grad, B.stream_handle(stream))

    def zero_grads(self, like_params):
        return {k: torch.zeros_like(t) for k, t in zip(("means", "log_scales", "quats", "opacity_logit", "rgb"),
                                                       like_params)}

    def patch_scale(self, Xr, Xp, patch, mask=None, stream=None):
        dev = Xr.device
        scale = torch.empty(self.win.n_patches(patch), device=dev)
        count = torch.empty(self.win.n_patches(patch), dtype=torch.int32, device=dev)
        B.patch_scale_align(self.win.c(), Xr, Xp, mask, patch, scale, count, B.stream_handle(stream))
        return scale, count

    def window_loss_into(self, rgb, target, pm, Xp, patch, alpha, scale, loss, grad_rgb, grad_pm, stream=None):
        B.window_loss(self.ctx, self.win.c(), rgb, target, pm, Xp, patch, alpha, scale, loss, grad_rgb, grad_pm,
                      B.stream_handle(stream))

    # -- scale alignment and pointmap replacement -----------------------------------------
    def new_align_result(self):
        return torch.empty(B.ALIGN_RESULT_DTYPE.itemsize * self.win.n_views, dtype=torch.uint8,
                           device=self.win.T_cw.device)

    def align_scale_into(self, Xr, Xp, result, mask=None, cfg: B.AlignConfig | None = None, stream=None):
        """Patch-based scale alignment of the prior Xp to the rendered Xr, every view."""
        cfg = cfg or B.AlignConfig()
        B.align_scale(self.ctx, self.win.c(), Xr, Xp, mask, cfg.c(), result, B.stream_handle(stream))

    def replace_pointmap_into(self, Xr, Xp, result, Xr_hat, replaced, eps_m=0.15, stream=None):
        """Eq. 14 with the aligned prior result[v].scale * Xp."""
        B.replace_pointmap(self.win.c(), Xr, Xp, result, eps_m, Xr_hat, replaced, B.stream_handle(stream))


    # -- regulariser and keyframe window ---------------------------------------------------
    def iso_loss_into(self, params, weight, loss, grad_log_scales=None, stream=None):
        """Eq. 16 times weight into loss [1]; its gradient is added to grad_log_scales."""
        B.iso_loss(self.ctx, _params(params), weight, loss, grad_log_scales, B.stream_handle(stream))

    def covisibility(self, frame_state, stream=None):
        """(iou [V][V], oc [V][V], visible counts [V]) of a forward run with mark_visible."""
        V = self.win.n_views
        dev = self.win.T_cw.device
        iou = torch.empty(V, V, dtype=torch.float64, device=dev)
        oc = torch.empty_like(iou)
        cnt = torch.empty(V, dtype=torch.int64, device=dev)
        B.covisibility(self.ctx, self.win.c(), self.n, frame_state, iou, oc, cnt, B.stream_handle(stream))
        return iou, oc, cnt

    def median_depth(self, depth, stream=None):
        """Median positive depth of each view (packed depth planes) -> float32 [V]."""
        out = torch.empty(self.win.n_views, device=self.win.T_cw.device)
        B.median_depth(self.ctx, self.win.c(), depth, out, B.stream_handle(stream))
        return out


def align_results(result: torch.Tensor):
    """Host view of a device gspm_align_result array (synchronises)."""
    return result.cpu().numpy().view(B.ALIGN_RESULT_DTYPE)


class RasterizePointmap(torch.autograd.Function):
    """Differentiable render of a window: (means, log_scales, quats, opacity_logit, rgb,
    xi) -> packed (rgb, depth, alpha, pointmap).

    ``xi`` [V][6] is the left se(3) perturbation of each pose (rho first); the forward
    renders at the window's poses T_cw and the pose gradient returned for ``xi`` is
    d L / d xi at xi = 0, so callers keep xi at zero and fold pose updates into T_cw with
    ``binding.pose_retract`` (Exp(xi) T_cw).

    With ``check`` False the forward does not synchronise: it renders with the
    Rasterizer's current pair capacity, and the overflow flag stays in the frame state
    until ``rast.check()`` reads it after the step.  A backward on an overflowed frame
    computes nothing (the library refuses it on the device), so the forward and its
    backward can be captured in one graph.  With ``check`` True the forward synchronises
    and re-renders with a larger capacity on overflow (eager use only)."""

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logit, rgb, xi, rast: Rasterizer, check: bool = False):
        params = (means.detach(), log_scales.detach(), quats.detach(), opacity_logit.detach(), rgb.detach())
        if check:
            out, fs = rast.forward(params)
        else:
            out = rast.new_outputs()
            fs = rast.new_frame_state()
            rast.forward_into(params, out, fs)
        rast.last_frame = fs
        ctx.rast = rast
        ctx.fs = fs
        ctx.save_for_backward(*params, out["rgb"], out["depth"], out["alpha"], out["pointmap"])
        ctx.want_pose = xi is not None and xi.requires_grad
        return out["rgb"], out["depth"], out["alpha"], out["pointmap"]

    @staticmethod
    def backward(ctx, g_rgb, g_depth, g_alpha, g_pm):
        *params, o_rgb, o_depth, o_alpha, o_pm = ctx.saved_tensors
        rast: Rasterizer = ctx.rast
        fwd = {"rgb": o_rgb, "depth": o_depth, "alpha": o_alpha, "pointmap": o_pm}
        up = {k: (v.contiguous() if v is not None else None)
              for k, v in (("rgb", g_rgb), ("depth", g_depth), ("alpha", g_alpha), ("pointmap", g_pm))}
        grads = {k: torch.empty_like(t) for k, t in zip(("means", "log_scales", "quats", "opacity_logit", "rgb"),
                                                          params)}
        pose = torch.empty(rast.win.n_views, 6, device=o_rgb.device) if ctx.want_pose else None
        rast.backward_into(params, fwd, up, ctx.fs, grads, pose, overwrite=True)
        return (grads["means"], grads["log_scales"], grads["quats"], grads["opacity_logit"], grads["rgb"], pose, None,
                None)


def rasterize(rast: Rasterizer, means, log_scales, quats, opacity_logit, rgb, xi=None, check=False):
    return RasterizePointmap.apply(means, log_scales, quats, opacity_logit, rgb, xi, rast, check)


class MappingStep:
    """One mapping iteration over a window, as a fixed launch sequence:

    render all views -> per-patch scale refit + L1 RGB / L1 pointmap loss gradient ->
    backward to every Gaussian parameter and every pose.

    Buffers are allocated once; ``run`` issues the launches eagerly, ``capture`` records
    them into a CUDA (HIP) graph that ``replay`` launches with one call.  Poses live in
    ``win.T_cw`` on the device, so in-place pose updates are seen by replays.  The pair
    capacity is fixed at capture time; ``check`` reads the forward's overflow flag."""

    def __init__(self, rast: Rasterizer, params, target_rgb, prior_pm, patch=8, alpha=0.98):
        self.rast = rast
        self.params = params
        self.target = target_rgb
        self.prior = prior_pm
        self.patch = patch
        self.alpha = alpha
        win = rast.win
        dev = win.T_cw.device
        self.out = rast.new_outputs()
        self.fs = rast.new_frame_state()
        self.scale = torch.empty(win.n_patches(patch), device=dev)
        self.loss = torch.empty(win.n_views, device=dev)
        self.g_rgb = torch.empty(3 * win.n_pixels, device=dev)
        self.g_pm = torch.empty(3 * win.n_pixels, device=dev)
        self.grads = rast.zero_grads(params)
        self.pose_grad = torch.zeros(win.n_views, 6, device=dev)
        rast.reserve()
        self.graph = None

    def run(self, stream=None):
        r = self.rast
        r.forward_into(self.params, self.out, self.fs, stream)
        r.window_loss_into(self.out["rgb"], self.target, self.out["pointmap"], self.prior, self.patch, self.alpha,
                           self.scale, self.loss, self.g_rgb, self.g_pm, stream)
        r.backward_into(self.params, self.out, {"rgb": self.g_rgb, "pointmap": self.g_pm}, self.fs, self.grads,
                        self.pose_grad, stream, overwrite=True)

    def check(self):
        return B.frame_status(self.fs, B.stream_handle())

    def capture(self):
        # Warm up on a side stream (allocator, first-launch costs), then record.
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        return self.graph

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()


class AutogradMappingStep:
    """One mapping iteration driven by torch.autograd: the window is rendered through
    ``RasterizePointmap`` from leaf tensors (the Gaussian parameters and a zero se(3)
    increment per pose), the library's window-loss kernel refits the per-patch scale and
    writes the loss and its image gradients, and ``torch.autograd.backward`` takes them
    through the function's backward into the leaves' ``.grad``.  Nothing synchronises, so
    ``capture`` records the whole step (forward, loss, backward) in one graph; ``check``
    reads the forward's overflow flag afterwards."""

    def __init__(self, rast: Rasterizer, params, target_rgb, prior_pm, patch=8, alpha=0.98):
        self.rast = rast
        self.leaves = [p.detach().clone().requires_grad_(True) for p in params]
        win = rast.win
        dev = win.T_cw.device
        self.xi = torch.zeros(win.n_views, 6, device=dev, requires_grad=True)
        self.target = target_rgb
        self.prior = prior_pm
        self.patch = patch
        self.alpha = alpha
        self.scale = torch.empty(win.n_patches(patch), device=dev)
        self.loss = torch.empty(win.n_views, device=dev)
        self.g_rgb = torch.empty(3 * win.n_pixels, device=dev)
        self.g_pm = torch.empty(3 * win.n_pixels, device=dev)
        rast.reserve()
        self.graph = None

    def run(self):
        for t in (*self.leaves, self.xi):
            t.grad = None
        rgb, _, _, pm = rasterize(self.rast, *self.leaves, self.xi)
        self.rast.window_loss_into(rgb.detach(), self.target, pm.detach(), self.prior, self.patch, self.alpha,
                                   self.scale, self.loss, self.g_rgb, self.g_pm)
        torch.autograd.backward([rgb, pm], [self.g_rgb, self.g_pm])

    def grads(self):
        names = ("means", "log_scales", "quats", "opacity_logit", "rgb")
        g = {k: t.grad for k, t in zip(names, self.leaves)}
        g["pose"] = self.xi.grad
        return g

    def check(self):
        return self.rast.check()

    def capture(self):
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.check()
        for t in (*self.leaves, self.xi):
            t.grad = None
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.run()
        return self.graph

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
