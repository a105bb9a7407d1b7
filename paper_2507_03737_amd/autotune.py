"""Autotuner for the batched mapping iteration.

The launch shape of the raster kernels (tile edge and pixels per lane, which together fix
the number of records staged per LDS batch: tile^2 / pixels_per_lane) and the radix digit
width trade binning and sorting cost against per-pixel work, and the best choice depends
on the window (view sizes, Gaussian count, footprint sizes).  ``autotune`` times whole
mapping iterations (render, patch scale + loss, backward) of every candidate on the
caller's own data and returns the fastest configuration.  Choices are cached in a JSON
file keyed by device, window geometry, Gaussian count and pointmap frame.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import torch

from . import binding as B
from .render import MappingStep, Rasterizer, Window

__all__ = ["Candidate", "default_candidates", "autotune", "cache_key"]

Candidate = Tuple[int, int, int]  # (tile, pixels_per_lane, sort_digit_bits)


def default_candidates(digit_bits: Sequence[int] = (6, 7, 8)) -> List[Candidate]:
    """Every supported raster shape with each digit width."""
    return [(t, p, d) for (t, p) in B.RasterConfig.SHAPES for d in digit_bits]


def cache_key(win: Window, n_gaussians: int, cfg: B.RasterConfig) -> str:
    dev = torch.cuda.get_device_name(win.T_cw.device)
    views = ";".join(f"{w}x{h}" for (h, w) in win.sizes)
    return f"{dev}|{views}|n={n_gaussians}|frame={cfg.pointmap_frame}"


def _load_cache(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def _store_cache(path: Optional[str], key: str, entry: dict) -> None:
    if not path:
        return
    data = _load_cache(path)
    data[key] = entry
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time_ms(fn, steps: int, warmup: int) -> float:
    for _ in range(warmup):
        fn()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def _sized_step(win, n, cfg, params, target, prior) -> MappingStep:
    """A mapping step whose pair capacity fits this configuration (30% headroom)."""
    rast = Rasterizer(win, n, cfg)
    probe = MappingStep(rast, params, target, prior)
    probe.run()
    try:
        pairs = probe.check()
    except B.CapacityError as e:
        pairs = e.pairs
    del probe
    rast.max_pairs = int(pairs * 1.3) + 4096
    step = MappingStep(rast, params, target, prior)
    step.run()
    step.check()
    return step


def autotune(win: Window, n_gaussians: int, params, target_rgb: torch.Tensor, prior_pm: torch.Tensor,
             base: Optional[B.RasterConfig] = None, candidates: Optional[Iterable[Candidate]] = None,
             steps: int = 5, warmup: int = 2, cache_path: Optional[str] = None,
             log=None, refine: int = 3, refine_steps: int = 20) -> Tuple[B.RasterConfig, List[dict]]:
    """Return the fastest configuration for this window, and the per-candidate timings.

    ``base`` supplies every setting that is not tuned (thresholds, pointmap frame).  Every
    candidate is timed over ``steps`` iterations, then the ``refine`` fastest over
    ``refine_steps``.  With ``cache_path`` a previous choice for the same key is returned
    without timing."""
    base = base or B.RasterConfig()
    key = cache_key(win, n_gaussians, base)
    hit = _load_cache(cache_path).get(key)
    if hit is not None:
        cfg = dataclasses.replace(base, tile=hit["tile"], pixels_per_lane=hit["pixels_per_lane"],
                                  sort_digit_bits=hit["sort_digit_bits"])
        return cfg, hit.get("results", [])
    results = []
    for (tile, ppl, bits) in (candidates if candidates is not None else default_candidates()):
        cfg = dataclasses.replace(base, tile=tile, pixels_per_lane=ppl, sort_digit_bits=bits)
        step = _sized_step(win, n_gaussians, cfg, params, target_rgb, prior_pm)
        ms = _time_ms(step.run, steps, warmup)
        step.check()
        results.append({"tile": tile, "pixels_per_lane": ppl, "sort_digit_bits": bits, "ms": ms})
        if log:
            log(f"[autotune] tile={tile} ppl={ppl} digit_bits={bits}: {ms:.3f} ms")
        del step
    # The short timings above separate the shapes; the few fastest candidates, often
    # within noise of each other, are timed again over more steps before choosing.
    finalists = sorted(results, key=lambda r: r["ms"])[:refine]
    best = None
    for r in finalists:
        cfg = dataclasses.replace(base, tile=r["tile"], pixels_per_lane=r["pixels_per_lane"],
                                  sort_digit_bits=r["sort_digit_bits"])
        if len(finalists) > 1:
            step = _sized_step(win, n_gaussians, cfg, params, target_rgb, prior_pm)
            r["ms_refined"] = _time_ms(step.run, refine_steps, warmup)
            step.check()
            del step
            if log:
                log(f"[autotune] refine tile={r['tile']} ppl={r['pixels_per_lane']} "
                    f"digit_bits={r['sort_digit_bits']}: {r['ms_refined']:.3f} ms")
        ms = r.get("ms_refined", r["ms"])
        if best is None or ms < best[0]:
            best = (ms, cfg)
    torch.cuda.empty_cache()
    cfg = best[1]
    _store_cache(cache_path, key, {"tile": cfg.tile, "pixels_per_lane": cfg.pixels_per_lane,
                                   "sort_digit_bits": cfg.sort_digit_bits, "results": results})
    return cfg, results
