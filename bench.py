"""Benchmark: one batched mapping iteration of the Gaussian pointmap rasterizer on MI355X.

Workload (default ``c3``): 1M Gaussians seen from a window of 8 keyframes of uneven size
(3 x 960x640, 3 x 1216x352, 2 x 640x480) along a synthetic driving trajectory.  One step
is the whole hot path over the window: project + depth sort + tile binning + forward
compositing of RGB / depth / alpha / camera-frame pointmap for all 8 views in one
global tile space, the per-8x8-patch least-squares scale refit and L1 RGB + L1 pointmap
loss gradient (alpha = 0.98), and the backward to every Gaussian parameter and all 8
poses.  The optimiser step is not part of it.

Inputs are synthetic and already resident on the GPU when timing starts: the optimised
map is the generated map G* perturbed by N(0, 0.05) on means and colours; the RGB
targets are renders of G*; the prior pointmap is the camera-frame pointmap of G* times a
per-8x8-patch scale U[0.8, 1.25] plus N(0, 0.02 m) noise.

Prints one JSON line.  ``value`` is Gaussian-pixel evaluations per second of the batched
step (contributing fragments of the forward plus the same fragments in the backward,
divided by the step time).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd ms/mapping iter & Gaussian-px evals/s, batched vs per-view, at oracle tol"

# Algorithmic work per contributing fragment, counted on the definition's operations with a
# fused multiply-add as two flops (the convention of the peak figure): 29 in the forward
# (the exponent, exp, the alpha clamp, 1 - alpha, the transmittance update, the weight and 7
# weighted accumulations) and 64 in the backward (recomputation, the dL/dalpha formula and
# the 13 gradient terms); the exponential counts as one.
FWD_FLOPS_PER_FRAG = 29
BWD_FLOPS_PER_FRAG = 64
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# Measured HBM traffic of the dominant kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by
# the same counters on a copy of known size) and the hash of the sources it was taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "raster_bwd_c3_traffic.txt")
# HBM bytes of a whole mapping iteration of the large window (sum over its kernels).
STEP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "mapping_step_c4_traffic.txt")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "raster_c3_counters.md")
KERNEL_SOURCES = ("paper_2507_03737_amd/csrc/raster.hip", "paper_2507_03737_amd/csrc/gspm_common.h")
COPY_BYTES = 1 << 29  # 512 MiB read + 512 MiB written by the calibration copy


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_inputs(name, seed, torch, dev):
    from paper_2507_03737_amd import scenes
    from paper_2507_03737_amd.render import Rasterizer, Window
    from paper_2507_03737_amd import binding as B

    sc = scenes.make_scene(name, seed=seed)
    rng = np.random.default_rng(1000 + seed)
    gt = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in sc.params()]
    means = sc.means + rng.normal(0.0, 0.05, sc.means.shape).astype(np.float32)
    rgb = sc.rgb + rng.normal(0.0, 0.05, sc.rgb.shape).astype(np.float32)
    opt = [torch.from_numpy(np.ascontiguousarray(a)).to(dev)
           for a in (means, sc.log_scales, sc.quats, sc.opacity_logit, rgb)]
    T = torch.from_numpy(np.ascontiguousarray(sc.T_cw)).to(dev)
    win = Window(sc.cams, T)
    cfg = B.RasterConfig(pointmap_frame=1)
    r_gt = Rasterizer(win, sc.n, cfg)
    out, _ = r_gt.forward(gt)
    target = out["rgb"].clone()
    # Prior: camera-frame pointmap of G* x per-8x8-patch scale + noise.
    g = torch.Generator(device=dev)
    g.manual_seed(2000 + seed)
    prior = torch.empty_like(out["pointmap"])
    for v, (h, w) in enumerate(win.sizes):
        ph, pw = math.ceil(h / 8), math.ceil(w / 8)
        s = torch.rand(ph, pw, device=dev, generator=g) * 0.45 + 0.8
        s = s.repeat_interleave(8, 0).repeat_interleave(8, 1)[:h, :w]
        seg = slice(3 * win.pix_off[v], 3 * win.pix_off[v + 1])
        pm = out["pointmap"][seg].view(3, h, w)
        prior[seg] = (pm * s[None] + 0.02 * torch.randn(3, h, w, device=dev, generator=g)).reshape(-1)
    del r_gt
    return sc, win, cfg, opt, target, prior


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def all_kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2507_03737_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def stored_record(path, kernel, workload, tile, ppl):
    """The machine-readable line of a committed counter summary, if it was taken on the
    current kernel sources and the same launch shape; else None."""
    try:
        with open(path) as fh:
            rec = json.loads([ln for ln in fh.read().splitlines() if ln.startswith("{")][-1])
    except (OSError, ValueError, IndexError):
        return None
    if (rec.get("kernel"), rec.get("workload"), rec.get("tile"), rec.get("ppl")) != (kernel, workload, tile, ppl):
        return None
    if rec.get("source_sha256") not in (kernel_source_hash(), all_kernel_sources_hash()):
        return None
    return rec


def stored_traffic(kernel, workload, tile, ppl):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy)."""
    rec = stored_record(TRAFFIC_FILE, kernel, workload, tile, ppl)
    return None if rec is None else rec.get("hbm_bytes_per_launch")


def copy_calibration(torch, dev):
    """A plain copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    n = COPY_BYTES // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log(f"[bench] calibration copy: 3 launches, {COPY_BYTES} bytes read and {COPY_BYTES} written each")
    del src, dst


def time_ms(fn, reps, torch):
    """Average milliseconds of fn over reps launches on the current stream (after 2 warm-ups)."""
    for _ in range(2):
        fn()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def time_mapping_ops(rast, step, win, sc, opt, cfg, torch, dev, reps=20):
    """Milliseconds and HBM rates of the mapping-side operations on the same window: scale
    alignment and pointmap replacement of the prior against the rendered pointmap, the
    isotropic regulariser, keyframe covisibility, median depth, and RANSAC + PnP between two
    views of the window (20k correspondences from the rendered pointmap, 20% outliers)."""
    import dataclasses
    from paper_2507_03737_amd import binding as B
    from paper_2507_03737_amd.render import Rasterizer
    from paper_2507_03737_amd.tracking import PnpConfig, draw_samples, pnp_ransac

    P = win.n_pixels
    R = sc.n * win.n_views
    out = {}
    pm, prior = step.out["pointmap"], step.prior
    res = rast.new_align_result()
    ms = time_ms(lambda: rast.align_scale_into(pm, prior, res), reps, torch)
    out["align_scale"] = {"ms": ms, "GB/s": 24 * P / (ms * 1e-3) / 1e9, "bytes": "24 B/px (Xr, Xp read once)"}
    hat = torch.empty_like(pm)
    rep = torch.empty(win.n_views, dtype=torch.int32, device=dev)
    ms = time_ms(lambda: rast.replace_pointmap_into(pm, prior, res, hat, rep), reps, torch)
    out["replace_pointmap"] = {"ms": ms, "GB/s": 36 * P / (ms * 1e-3) / 1e9, "bytes": "24 B/px read + 12 B/px written"}
    loss = torch.empty(1, device=dev)
    g = torch.zeros(3, sc.n, device=dev)
    ms = time_ms(lambda: rast.iso_loss_into(opt, 10.0, loss, g), reps, torch)
    out["iso_loss"] = {"ms": ms, "GB/s": 36 * sc.n / (ms * 1e-3) / 1e9,
                       "bytes": "12 B/Gaussian read + 12 B/Gaussian gradient read and written"}
    rv = Rasterizer(win, sc.n, dataclasses.replace(cfg, mark_visible=1))
    rv.max_pairs = rast.max_pairs
    o, fs = rv.forward(opt)
    ms = time_ms(lambda: rv.covisibility(fs), reps, torch)
    out["covisibility"] = {"ms": ms, "GB/s": R / (ms * 1e-3) / 1e9, "bytes": "1 B/record"}
    del rv, o, fs
    ms = time_ms(lambda: rast.median_depth(step.out["depth"]), reps, torch)
    out["median_depth"] = {"ms": ms, "GB/s": 4 * P / (ms * 1e-3) / 1e9, "bytes": "4 B/px"}
    # PnP: view 0's rendered points seen from view 1 (true relative pose), 1 px noise, 20% outliers.
    h0, w0 = win.sizes[0]
    X0 = step.out["pointmap"][:3 * h0 * w0].view(3, -1)
    A = step.out["alpha"][:h0 * w0]
    gen = torch.Generator(device=dev)
    gen.manual_seed(77)
    idx = torch.nonzero(A > 0.5).flatten()
    idx = idx[torch.randperm(idx.numel(), device=dev, generator=gen)[:20000]]
    X = X0[:, idx].contiguous()
    T0 = win.T_cw[0].double().view(3, 4)
    T1 = win.T_cw[1].double().view(3, 4)
    Rr = T1[:, :3] @ T0[:, :3].T
    tr = T1[:, 3] - Rr @ T0[:, 3]
    Y = Rr @ X.double() + tr[:, None]
    c1 = win.cams[1]
    uv = torch.stack([c1.fx * Y[0] / Y[2] + c1.cx, c1.fy * Y[1] / Y[2] + c1.cy])
    uv = uv + torch.randn(uv.shape, device=dev, generator=gen, dtype=torch.float64)
    bad = torch.rand(uv.shape[1], device=dev, generator=gen) < 0.2
    uv[:, bad] += 50.0 + 100.0 * torch.rand((2, int(bad.sum())), device=dev, generator=gen, dtype=torch.float64)
    uv = uv.float().contiguous()
    pcfg = PnpConfig(n_hypotheses=1024, threshold=3.0)
    samples = draw_samples(X.shape[1], pcfg.n_hypotheses, generator=gen, device=dev)
    ctx = B.Context()
    ms = time_ms(lambda: pnp_ransac(X, uv, c1, samples, pcfg, ctx=ctx), 5, torch)
    T, cnt, _, _, _ = pnp_ransac(X, uv, c1, samples, pcfg, ctx=ctx)
    err_t = float(torch.linalg.norm(T[:, 3] - tr).item())
    out["pnp_ransac"] = {"ms": ms, "correspondences": int(X.shape[1]), "hypotheses": pcfg.n_hypotheses,
                         "inliers": int(cnt.item()), "translation_error_m": err_t}
    return out


def time_tracking(torch, dev, iters=20):
    """ms per tracking iteration on the tracking configuration (500k Gaussians, one 960x640
    view, pose perturbed by 2 deg / 0.3 m): render, L1 RGB + L1 pointmap loss gradient,
    pose-only backward (Sec. 3.2.2, Eq. 10-11)."""
    from paper_2507_03737_amd import scenes
    from paper_2507_03737_amd import binding as B
    from paper_2507_03737_amd.render import Rasterizer, Window
    sc = scenes.make_scene("c2")
    params = [torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in sc.params()]
    cfg = B.RasterConfig(pointmap_frame=1)
    T_true = torch.from_numpy(np.ascontiguousarray(sc.T_cw)).to(dev)
    out_t, _ = Rasterizer(Window(sc.cams, T_true), sc.n, cfg).forward(params)
    T = torch.from_numpy(np.ascontiguousarray(scenes.perturb_pose(sc.T_cw[0], 2.0, 0.3, 2)[None])).to(dev)
    win = Window(sc.cams, T)
    rast = Rasterizer(win, sc.n, cfg)
    rast.forward(params)
    rast.max_pairs = int(rast.pairs * 1.5) + 4096
    out, fs = rast.new_outputs(), rast.new_frame_state()
    scale = torch.empty(win.n_patches(8), device=dev)
    loss = torch.empty(1, device=dev)
    g_rgb, g_pm = torch.empty_like(out["rgb"]), torch.empty_like(out["pointmap"])
    pose = torch.zeros(1, 6, device=dev)
    rast.reserve()

    def it():
        rast.forward_into(params, out, fs)
        rast.window_loss_into(out["rgb"], out_t["rgb"], out["pointmap"], out_t["pointmap"], 8, 0.98, scale, loss,
                              g_rgb, g_pm)
        pose.zero_()
        rast.pose_backward_into(params, out, {"rgb": g_rgb, "pointmap": g_pm}, fs, pose)
    ms, _ = time_steps(it, iters, 3, torch)
    B.frame_status(fs, B.stream_handle())
    return {"workload": "500k Gaussians, one 960x640 view, pose-only backward", "ms_per_iter": ms}


def time_steps(fn, steps, warmup, torch, stats=None):
    """Mean milliseconds per step over `steps` steps bracketed by synchronisations (one
    event pair around all of them), and the wall time.  With a dict `stats`, each step is
    also bracketed by its own event pair and the dict receives the per-step median, p10
    and p90."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if stats is not None else None
    w0 = time.perf_counter()
    t0.record()
    for k in range(steps):
        if marks:
            marks[k].record()
        fn()
    if marks:
        marks[steps].record()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    if marks:
        per = np.array([marks[k].elapsed_time(marks[k + 1]) for k in range(steps)])
        stats.update({"median": float(np.median(per)), "p10": float(np.percentile(per, 10)),
                      "p90": float(np.percentile(per, 90)), "steps": steps})
    return t0.elapsed_time(t1) / steps, wall


def gpu_clocks():
    """Current shader and memory clocks as rocm-smi reports them (None if unavailable)."""
    import subprocess
    try:
        r = subprocess.run(["rocm-smi", "--showclocks"], capture_output=True, text=True, timeout=20)
    except (OSError, subprocess.SubprocessError):
        return None
    lines = [ln.strip() for ln in r.stdout.splitlines() if "clock level" in ln and ("sclk" in ln or "mclk" in ln)]
    return lines or None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(sc, opt_host, win_cams, T_host, seed, budget_px):
    """Oracle forward + backward on a bounded sample of pixel crops of the same window:
    32x32 crops spread evenly over the views (each view projected once)."""
    from oracle import oracle as O

    O.build()
    p = O.Params(*opt_host)
    S = O.Settings()
    rng = np.random.default_rng(seed)
    views = len(win_cams)
    crop = 32
    per_view = max(1, budget_px // (crop * crop * views))
    frags = 0
    npx = 0
    t0 = time.perf_counter()
    for v in range(views):
        cam = win_cams[v]
        boxes = []
        for _ in range(per_view):
            x0 = int(rng.integers(0, cam.width - crop))
            y0 = int(rng.integers(0, cam.height - crop))
            boxes.append((x0, y0, crop, crop))
        pix = np.concatenate([O.crop_pixels(*b) for b in boxes])
        pix = np.ascontiguousarray(np.unique(pix[:, [1, 0]], axis=0)[:, [1, 0]], dtype=np.int32)
        view = O.make_view(cam, T_host[v])
        proj = O.project(p, view, S)
        r = O.render(p, view, S, pix, proj=proj)
        up = {"rgb": np.ones((pix.shape[0], 3)), "depth": np.zeros(pix.shape[0]),
              "alpha": np.zeros(pix.shape[0]), "pointmap": np.ones((pix.shape[0], 3))}
        O.backward(p, view, S, pix, up, pointmap_frame=1, proj=proj)
        frags += int(r["n_frag"].sum())
        npx += pix.shape[0]
    dt = time.perf_counter() - t0
    return {"value": 2.0 * frags / dt, "unit": "Gaussian-px evals/s", "cores": O.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{per_view} crops of {crop}x{crop} px per view ({npx} px) over the {views} views, FP64 "
                      f"projection + forward + backward (OpenMP), {frags} contributing fragments, {dt:.1f} s"}


def cpu_baseline_c0_one_thread():
    """The oracle's full-frame forward + backward of the small configuration (2,000
    Gaussians, 160x120) on one thread."""
    from oracle import oracle as O
    from paper_2507_03737_amd import scenes

    O.build()
    sc = scenes.make_scene("c0")
    p = O.Params.from_scene(sc)
    S = O.Settings()
    cam = sc.cams[0]
    view = O.make_view(cam, sc.T_cw[0])
    pix = O.full_pixels(cam)
    up = O.pixel_upstream(scenes.upstream_grads(sc, seed=1)[0], pix)
    n0 = O.num_threads()
    O.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        proj = O.project(p, view, S)
        r = O.render(p, view, S, pix, proj=proj)
        O.backward(p, view, S, pix, up, pointmap_frame=1, proj=proj)
        dt = time.perf_counter() - t0
    finally:
        O.set_num_threads(n0)
    frags = int(r["n_frag"].sum())
    return {"value": 2.0 * frags / dt, "unit": "Gaussian-px evals/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"c0 full frame (2,000 Gaussians, 160x120), FP64 forward + backward, {frags} contributing "
                      f"fragments, {dt:.2f} s"}


def sized_step(rast, opt, target, prior, MappingStep, B):
    """A mapping step whose pair capacity fits the window with 30% headroom."""
    probe = MappingStep(rast, opt, target, prior)
    probe.run()
    try:
        pairs = probe.check()
    except B.CapacityError as e:
        pairs = e.pairs
    del probe
    rast.max_pairs = int(pairs * 1.3) + 4096
    return MappingStep(rast, opt, target, prior)


def time_autograd_step(rast, opt, target, prior, steps, warmup, torch):
    """The same mapping iteration driven by torch.autograd (render through the autograd
    function, window loss, torch.autograd.backward into the leaves), eager and as one
    captured graph."""
    from paper_2507_03737_amd.render import AutogradMappingStep
    step = AutogradMappingStep(rast, opt, target, prior)
    st_e, st_g = {}, {}
    ms_e, _ = time_steps(step.run, steps, warmup, torch, st_e)
    step.check()
    ms_g = None
    try:
        step.capture()
        ms_g, _ = time_steps(step.replay, steps, 2, torch, st_g)
        step.check()
    except Exception as e:  # report eager only
        log(f"[bench] autograd step capture failed: {e}")
    del step
    return {"eager_ms": ms_e, "eager_stats": st_e, "graph_ms": ms_g, "graph_stats": st_g or None}


def large_window(steps, warmup, torch, dev):
    """The large window (16 keyframes of 1920x1080, 3M Gaussians): autotuned ms per mapping
    iteration with per-pixel transmittance recomputed in the backward (8 bytes of state per
    pixel), its HBM traffic from the committed counter summary of this launch shape (when
    it was taken on the current kernel sources), and the device memory the window uses."""
    from paper_2507_03737_amd import binding as B
    from paper_2507_03737_amd.autotune import autotune
    from paper_2507_03737_amd.render import MappingStep, Rasterizer

    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats(dev)
    free0, _ = torch.cuda.mem_get_info(dev)
    log("[bench] building c4 inputs")
    sc, win, cfg, opt, target, prior = build_inputs("c4", 4, torch, dev)
    cfg, tuned = autotune(win, sc.n, opt, target, prior, base=cfg,
                          candidates=[(16, 1, 8), (16, 2, 8), (32, 1, 8), (32, 2, 8)], steps=3, warmup=1,
                          refine=2, refine_steps=8, log=log)
    rast = Rasterizer(win, sc.n, cfg)
    step = sized_step(rast, opt, target, prior, MappingStep, B)
    rast.cfg.count_work = 1
    step.run()
    pairs, frags = rast.work(step.fs)[:2]
    rast.cfg.count_work = 0
    st = {}
    rast.ctx.timing(True)
    ms, _ = time_steps(step.run, steps, warmup, torch, st)
    phases = rast.ctx.collect_timing()
    rast.ctx.timing(False)
    step.check()
    st_g = {}
    ms_g = None
    try:
        step.capture()
        ms_g, _ = time_steps(step.replay, steps, 2, torch, st_g)
        step.check()
    except Exception as e:
        log(f"[bench] c4 graph capture failed: {e}")
    free1, _ = torch.cuda.mem_get_info(dev)
    n_iter = max(1, phases["raster_fwd"][1])
    rec = stored_record(STEP_TRAFFIC_FILE, "mapping_step", "c4", cfg.tile, cfg.pixels_per_lane)
    hbm = None
    if rec is not None:
        hbm = {"bytes_per_iter": rec["hbm_bytes_per_iter"], "GB/s": rec["hbm_bytes_per_iter"] / (ms * 1e-3) / 1e9,
               "frac": rec["hbm_bytes_per_iter"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    log(f"[bench] c4 {ms:.3f} ms/iter (tile {cfg.tile}, {cfg.pixels_per_lane} px/lane)")
    out = {"workload": "c4 large window: 3M Gaussians, 16 keyframes 1920x1080, render + patch-scale L1 loss + "
                       "backward to all params and poses, transmittance recomputed in the backward",
           "tile": cfg.tile, "pixels_per_lane": cfg.pixels_per_lane, "sort_digit_bits": cfg.sort_digit_bits,
           "autotune_ms": {f"{r['tile']}x{r['tile']}/ppl{r['pixels_per_lane']}": round(r.get("ms_refined", r["ms"]), 3)
                           for r in tuned},
           "ms_per_iter": ms, "stats": st, "graph_ms_per_iter": ms_g, "graph_stats": st_g or None,
           "tile_pairs": pairs, "contributing_fragments": frags, "gaussian_px_evals_per_s": 2.0 * frags / (ms * 1e-3),
           "phase_ms": {k: round(v[0] / n_iter, 4) for k, v in phases.items()},
           "hbm": hbm,
           "memory": {"device_used_bytes": int(free0 - free1),
                      "torch_peak_bytes": int(torch.cuda.max_memory_allocated(dev)),
                      "per_pixel_state_bytes": 12}}
    del step, rast, opt, target, prior
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4"])
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--tile", type=int, default=None, help="raster tile edge (default: autotuned)")
    ap.add_argument("--ppl", type=int, default=None, help="pixels per lane of the raster kernels (default: autotuned)")
    ap.add_argument("--digit-bits", type=int, default=None, help="radix digit width (default: autotuned)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-per-view", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--cpu-px", type=int, default=131072, help="pixels in the CPU-baseline sample")
    ap.add_argument("--no-extras", action="store_true", help="skip timing the mapping-side operations")
    ap.add_argument("--no-c4", action="store_true", help="skip the large-window (c4) leg")
    ap.add_argument("--no-autograd", action="store_true", help="skip the autograd-driven step")
    ap.add_argument("--no-clocks", action="store_true",
                    help="do not query clocks with rocm-smi (a child process; under a profiler that preloads "
                         "itself into children, its interpreter start is refused)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a copy of known size (for scaling HBM traffic counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; multi-GPU sharding is described in "
                                   "DESIGN.md but not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2507_03737_amd import binding as B
    from paper_2507_03737_amd.render import MappingStep, Rasterizer

    dev = torch.device("cuda:0")
    B.load()
    free0, total_mem = torch.cuda.mem_get_info(dev)
    if args.calibrate_copy:
        copy_calibration(torch, dev)
    seed = args.seed if args.seed is not None else ["c0", "c1", "c2", "c3", "c4"].index(args.workload)
    log(f"[bench] building {args.workload} inputs")
    sc, win, cfg, opt, target, prior = build_inputs(args.workload, seed, torch, dev)
    tuned = None
    if args.tile is None and args.ppl is None and args.digit_bits is None:
        from paper_2507_03737_amd.autotune import autotune
        cfg, tuned = autotune(win, sc.n, opt, target, prior, base=cfg, log=log)
        log(f"[bench] autotuned: tile={cfg.tile} ppl={cfg.pixels_per_lane} digit_bits={cfg.sort_digit_bits}")
    else:
        cfg.tile = args.tile if args.tile is not None else 16
        cfg.pixels_per_lane = args.ppl if args.ppl is not None else 1
        cfg.sort_digit_bits = args.digit_bits if args.digit_bits is not None else 8

    # ---- batched window -------------------------------------------------------------------
    rast = Rasterizer(win, sc.n, cfg)
    probe = MappingStep(rast, opt, target, prior)
    probe.run()
    try:
        pairs = probe.check()
    except B.CapacityError as e:
        pairs = e.pairs
    del probe
    rast.max_pairs = int(pairs * 1.3) + 4096
    step = MappingStep(rast, opt, target, prior)
    rast.cfg.count_work = 1  # one forward that also counts its contributing fragments
    step.run()
    pairs, frags, evals_bound, walked, accepted = rast.work(step.fs)
    rast.cfg.count_work = 0
    log(f"[bench] pairs={pairs} contributing fragments={frags}")

    clocks_before = None if args.no_clocks else gpu_clocks()
    stats = {"batched_eager": {}, "batched_graph": {}, "per_view_eager": {}}
    rast.ctx.timing(True)
    ms_batched, wall = time_steps(step.run, args.steps, args.warmup, torch, stats["batched_eager"])
    phases = rast.ctx.collect_timing()
    rast.ctx.timing(False)
    step.check()
    log(f"[bench] batched eager {ms_batched:.3f} ms/step")

    ms_graph = None
    if not args.no_graph:
        try:
            step.capture()
            ms_graph, _ = time_steps(step.replay, args.steps, 2, torch, stats["batched_graph"])
            step.check()
            log(f"[bench] batched graph {ms_graph:.3f} ms/step")
        except Exception as e:  # graph capture unsupported -> report eager only
            log(f"[bench] graph capture failed: {e}")

    # ---- per-view path: the same kernels, one view at a time, no graph ---------------------
    ms_per_view = None
    if not args.no_per_view:
        steps_v = []
        for v in range(win.n_views):
            sub = win.subwindow(v)
            r = Rasterizer(sub, sc.n, cfg)
            sl = slice(3 * win.pix_off[v], 3 * win.pix_off[v + 1])
            s_v = MappingStep(r, opt, target[sl].contiguous(), prior[sl].contiguous())
            s_v.run()
            try:
                need = s_v.check()
            except B.CapacityError as e:
                need = e.pairs
            r.max_pairs = int(need * 1.3) + 4096
            s_v = MappingStep(r, opt, target[sl].contiguous(), prior[sl].contiguous())
            steps_v.append(s_v)

        def per_view():
            for s_v in steps_v:
                s_v.run()
        ms_per_view, _ = time_steps(per_view, args.steps, args.warmup, torch, stats["per_view_eager"])
        log(f"[bench] per-view eager {ms_per_view:.3f} ms/step")
        del steps_v

    # ---- roofline of the dominant kernel ---------------------------------------------------
    # Phase time per iteration (a phase may be timed in several segments per iteration, as
    # binning is), and per timed segment for the dominant kernel's roofline.
    n_iter = max(1, phases["raster_fwd"][1])
    ph_iter = {k: v[0] / n_iter for k, v in phases.items()}
    ph_ms = {k: (v[0] / max(1, v[1])) for k, v in phases.items()}
    dominant = max(ph_iter, key=lambda k: ph_iter[k])
    if dominant in ("raster_fwd", "raster_bwd"):
        flops = frags * (FWD_FLOPS_PER_FRAG if dominant == "raster_fwd" else BWD_FLOPS_PER_FRAG)
        achieved = flops / (ph_ms[dominant] * 1e-3) / 1e12
        roof = {"kernel": dominant, "bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK_TFLOPS,
                "traffic": stored_traffic(dominant, args.workload, cfg.tile, cfg.pixels_per_lane),
                "algorithmic": f"{frags} contributing fragments x "
                               f"{FWD_FLOPS_PER_FRAG if dominant == 'raster_fwd' else BWD_FLOPS_PER_FRAG} flop"}
    else:
        # Sorting / streaming phases: algorithmic bytes = one read and one write of the data.
        nbytes = {"tile_sort": 16 * pairs, "depth_sort": 16 * sc.n * win.n_views,
                  "preprocess": (56 + 64) * sc.n * win.n_views, "binning": 12 * pairs,
                  "param_bwd": (56 + 64 + 56) * sc.n * win.n_views}[dominant]
        achieved = nbytes / (ph_iter[dominant] * 1e-3) / 1e9
        roof = {"kernel": dominant, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "algorithmic": f"{nbytes} bytes"}
    roof["kernel_ms"] = ph_ms[dominant]
    # Instruction issue: the counted wave-level VALU instructions per launch over this run's
    # launch time, against 1024 SIMDs x 2.4 GHz / 4 cycles per wave64 instruction.
    cnt = stored_record(COUNTERS_FILE, dominant, args.workload, cfg.tile, cfg.pixels_per_lane)
    if cnt is not None and "valu_insts_per_launch" in cnt:
        roof["valu_issue_frac"] = cnt["valu_insts_per_launch"] / (ph_ms[dominant] * 1e-3) / cnt["valu_issue_peak_per_s"]

    # At one pixel per lane the backward sums each record's values over a wave's pixels on
    # the matrix cores; the same step with the cross-lane reduce-scatter instead, for
    # comparison (same shape, same inputs).
    bwd_forms = None
    if cfg.pixels_per_lane == 1:
        rast.cfg.bwd_lane_reduce = 1
        rast.ctx.timing(True)
        ms_lane, _ = time_steps(step.run, args.steps, args.warmup, torch)
        ph_lane = rast.ctx.collect_timing()
        rast.ctx.timing(False)
        step.check()
        rast.cfg.bwd_lane_reduce = 0
        bwd_forms = {"matrix_cores": {"raster_bwd_ms": ph_ms["raster_bwd"], "step_ms": ms_batched},
                     "lane_reduce_scatter": {"raster_bwd_ms": ph_lane["raster_bwd"][0] / max(1, ph_lane["raster_bwd"][1]),
                                             "step_ms": ms_lane}}
        log(f"[bench] backward with the lane reduce-scatter: {bwd_forms['lane_reduce_scatter']['raster_bwd_ms']:.3f} ms")

    autograd = None
    if not args.no_autograd:
        log("[bench] autograd-driven step")
        autograd = time_autograd_step(Rasterizer(win, sc.n, cfg, max_pairs=rast.max_pairs), opt, target, prior,
                                      args.steps, args.warmup, torch)
        log(f"[bench] autograd step {autograd['eager_ms']:.3f} ms eager, {autograd['graph_ms']} ms graph")

    mapping_ops = None
    tracking = None
    if not args.no_extras:
        log("[bench] mapping-side operations")
        mapping_ops = time_mapping_ops(rast, step, win, sc, opt, cfg, torch, dev)
        log("[bench] tracking iteration")
        tracking = time_tracking(torch, dev)

    free1, _ = torch.cuda.mem_get_info(dev)
    memory = {"device_used_bytes": int(free0 - free1), "torch_peak_bytes": int(torch.cuda.max_memory_allocated(dev)),
              "device_total_bytes": int(total_mem)}
    clocks_after = None if args.no_clocks else gpu_clocks()

    c4 = None
    if not args.no_c4 and args.workload == "c3":
        del step, rast
        c4 = large_window(max(5, args.steps // 2), 2, torch, dev)

    cpu = cpu1 = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        opt_host = [t.cpu().numpy() for t in opt]
        cpu = cpu_baseline(sc, opt_host, sc.cams, sc.T_cw, 7, args.cpu_px)
        cpu1 = cpu_baseline_c0_one_thread()
    fps_evals = 2.0 * frags / (ms_batched * 1e-3)
    res = {
        "metric": METRIC,
        "value": fps_evals,
        "unit": "Gaussian-px evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batched,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": {"c1": "c1 single outdoor frame 1216x352, 300k Gaussians",
                         "c2": "c2 single frame 960x640, 500k Gaussians",
                         "c3": "c3 batched mapping window: 1M Gaussians, 8 keyframes (3x960x640, 3x1216x352, "
                               "2x640x480), render + patch-scale L1 loss + backward to all params and poses",
                         "c4": "c4 16 keyframes 1920x1080, 3M Gaussians"}[args.workload],
            "n_gaussians": sc.n, "views": [[c.width, c.height] for c in sc.cams], "tile": cfg.tile,
            "pixels_per_lane": cfg.pixels_per_lane, "sort_digit_bits": cfg.sort_digit_bits,
            "autotuned": tuned is not None,
            "patch": 8, "loss_alpha": 0.98, "pointmap_frame": "camera",
            "bwd_reduction": ("matrix cores: each wave's per-record sums as a v_mfma_f32_16x16x4f32 contraction "
                              "(the cross-lane DPP reduce-scatter form is timed beside it)"
                              if cfg.pixels_per_lane == 1 else "cross-lane DPP reduce-scatter"),
        },
        "fwd_bwd_ms_per_iter": {"batched_eager": ms_batched, "batched_graph": ms_graph, "per_view_eager": ms_per_view,
                                "batched_eager_lane_reduce_scatter": bwd_forms["lane_reduce_scatter"]["step_ms"]
                                if bwd_forms else None},
        "step_stats_ms": stats,
        "gpu_clocks": {"before": clocks_before, "after": clocks_after},
        "batched_speedup_vs_per_view": (ms_per_view / ms_batched) if ms_per_view else None,
        "work": {"tile_pairs": pairs, "contributing_fragments": frags, "evaluated_bound": evals_bound,
                 "fwd_walked_wave_entries": walked, "accepted_wave_entries": accepted,
                 "fwd_lane_evals_per_fragment": 64.0 * walked / max(1, frags),
                 "bwd_lane_evals_per_fragment": 64.0 * accepted / max(1, frags)},
        "phase_ms": {k: round(v, 4) for k, v in ph_iter.items()},
        "autotune_ms": ({f"{r['tile']}x{r['tile']}/ppl{r['pixels_per_lane']}/bits{r['sort_digit_bits']}": round(r["ms"], 3)
                         for r in tuned} if tuned else None),
        "autotune_refined_ms": ({f"{r['tile']}x{r['tile']}/ppl{r['pixels_per_lane']}/bits{r['sort_digit_bits']}":
                                 round(r["ms_refined"], 3) for r in tuned if "ms_refined" in r} if tuned else None),
        "roofline": roof,
        "bwd_reduction_forms": bwd_forms,
        "memory": memory,
        "cpu_baseline": cpu,
        "cpu_baseline_c0_one_thread": cpu1,
        "autograd_step": autograd,
        "c4": c4,
        "mapping_ops": mapping_ops,
        "tracking": tracking,
        "wall_s_timed": wall,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
