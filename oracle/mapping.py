"""FP64 oracle for the mapping-side steps around the rasterizer (numpy).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU-baseline leg,
never by the product path.  Every function is the plain statement of the step it names,
in double precision, with no blocking or reordering beyond what the statement implies.

* ``align_scale`` -- patch-based pointmap scale alignment (supplementary Alg. 1, the
  procedure behind Sec. 3.3.1, with the parameters of the supplementary parameter
  table: P = 10, delta_mu = delta_sigma = 0.3, eps_r = 0.1, max_iter = 3, tau = 0.01).
* ``replace_pointmap`` -- pointmap replacement (Sec. 3.3.2, Eq. 14, eps_m = 0.15).
* ``iso_loss`` -- isotropic regulariser (Sec. 3.3.3, Eq. 16) and its gradient.
* ``covisibility`` -- keyframe covisibility IOU and overlap coefficient (supplementary
  Eq. S1-S2) from per-view visibility sets.
* ``median_depth`` -- median of the positive rendered depths of a view (the median
  pointmap depth used by the keyframe rule of the supplementary keyframe management).

Readings where the text leaves a choice (each mirrored by the library):

* Alg. 1 compares statistics of pointmaps, which hold 3-vectors per pixel; the per-pixel
  scalar is the Euclidean norm |X(x)| (distance from the camera centre).  It scales with
  the pointmap, so the relative tests "< delta * mu_p" are well posed (a per-channel mean
  can be zero or negative).
* Means and standard deviations are over the valid pixels of a patch (mask nonzero;
  border patches are partial); the standard deviation is the population one.
* CP is empty at the start of every iteration; sigma' is computed once per iteration over
  the CP of all candidate patches (the last assignment inside the printed candidate loop
  sees the same set) and measures the original X^p: sigma' = mean|X^r[CP]| / mean|X^p[CP]|,
  so that X^p_{iter+1} = sigma' X^p does not compound.  An empty CP leaves sigma' as it
  was.  The loop runs exactly max_iter times.
* |CP| < tau N_p (N_p = valid pixels) flags the view for the scale remedy, which needs
  image matching and is not part of this library.
* Eq. 14 compares vectors through norms: X^r(x) is kept when
  |X^r(x) - Xp_hat(x)| <= eps_m |Xp_hat(x)|, and replaced by Xp_hat(x) otherwise.
* Eq. 16 uses the activated scales s = exp(log_scale) and sign(0) = 0.
* A Gaussian is visible in a keyframe when it contributes to at least one pixel of that
  keyframe's render.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# Supplementary Alg. 1: patch-based pointmap scale alignment.

def _patches(H, W, P):
    for py in range(-(-H // P)):
        for px in range(-(-W // P)):
            yield slice(py * P, min(H, (py + 1) * P)), slice(px * P, min(W, (px + 1) * P))


def align_scale(Xr, Xp, P=10, delta_mu=0.3, delta_sigma=0.3, eps_r=0.1, max_iter=3, tau=0.01, mask=None):
    """Scale sigma' that aligns the prior pointmap Xp to the rendered one Xr.

    Xr, Xp: [3][H][W]; mask: [H][W] (nonzero = valid) or None.  Returns a dict with
    ``scale`` (sigma'), ``cp`` (|CP| of the last iteration), ``n_valid`` (N_p),
    ``insufficient`` (|CP| < tau N_p), ``scales`` (sigma' after each iteration) and
    ``margin`` (the smallest distance of any candidate or CP decision from its threshold,
    relative to the threshold, over all iterations)."""
    Xr = np.asarray(Xr, dtype=np.float64)
    Xp = np.asarray(Xp, dtype=np.float64)
    _, H, W = Xr.shape
    valid = np.ones((H, W), bool) if mask is None else (np.asarray(mask) != 0)
    nr = np.sqrt((Xr * Xr).sum(axis=0))
    sigma = 1.0
    scales = []
    margin = np.inf
    cp_count = 0
    for _ in range(max_iter):
        Xp_it = sigma * Xp                               # X^p_iter
        np_it = np.sqrt((Xp_it * Xp_it).sum(axis=0))
        cand = []
        for sl in _patches(H, W, P):
            v = valid[sl]
            if not v.any():
                continue
            r, p = nr[sl][v], np_it[sl][v]
            mu_r, sd_r = r.mean(), r.std()
            mu_p, sd_p = p.mean(), p.std()
            t_mu, t_sd = delta_mu * mu_p, delta_sigma * sd_p
            ok = abs(mu_r - mu_p) < t_mu and abs(sd_r - sd_p) < t_sd
            if t_mu > 0:
                margin = min(margin, abs(abs(mu_r - mu_p) - t_mu) / t_mu)
            if t_sd > 0:
                margin = min(margin, abs(abs(sd_r - sd_p) - t_sd) / t_sd)
            if ok:
                cand.append((sl, mu_r, sd_r, mu_p, sd_p))
        cp = np.zeros((H, W), bool)
        for sl, mu_r, sd_r, mu_p, sd_p in cand:
            zr = (nr[sl] - mu_r) / sd_r                  # X^r_N
            zp = (np_it[sl] - mu_p) / sd_p               # X^p_N
            d = np.abs(zr - zp)
            sel = (d < eps_r) & valid[sl]
            cp[sl] |= sel
            if valid[sl].any():
                margin = min(margin, float((np.abs(d[valid[sl]] - eps_r) / eps_r).min()))
        cp_count = int(cp.sum())
        if cp_count > 0:
            np0 = np.sqrt((Xp * Xp).sum(axis=0))         # the original X^p
            sigma = nr[cp].mean() / np0[cp].mean()
        scales.append(sigma)
    n_valid = int(valid.sum())
    return {"scale": sigma, "cp": cp_count, "n_valid": n_valid, "insufficient": cp_count < tau * n_valid,
            "scales": scales, "margin": margin}


# ---------------------------------------------------------------------------
# Eq. 14: pointmap replacement.

def replace_pointmap(Xr, Xp, scale, eps_m=0.15):
    """Xr_hat = Xr where |Xr - s Xp| <= eps_m |s Xp|, else s Xp (per pixel, s = sigma').

    Returns (Xr_hat [3][H][W] float64, replaced mask [H][W], margin) where margin is the
    smallest |d - eps_m |Xp_hat|| relative to eps_m |Xp_hat| over the pixels."""
    Xr = np.asarray(Xr, dtype=np.float64)
    Xh = float(scale) * np.asarray(Xp, dtype=np.float64)
    d = np.sqrt(((Xr - Xh) ** 2).sum(axis=0))
    t = eps_m * np.sqrt((Xh * Xh).sum(axis=0))
    keep = d <= t
    out = np.where(keep[None], Xr, Xh)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.abs(d - t) / t
    margin = float(np.nanmin(np.where(t > 0, rel, np.inf))) if d.size else np.inf
    return out, ~keep, margin


# ---------------------------------------------------------------------------
# Eq. 16: isotropic regulariser.

def iso_loss(log_scales, weight=1.0):
    """weight * sum_i sum_k |s_ik - mean_k s_ik| with s = exp(log_scales) ([3][n]).

    Returns (loss, d loss / d log_scales [3][n])."""
    s = np.exp(np.asarray(log_scales, dtype=np.float64))
    m = s.mean(axis=0)
    r = s - m[None]
    sg = np.sign(r)
    loss = weight * np.abs(r).sum()
    # d|s_k - m| / d s_j = sg_k (delta_kj - 1/3)
    g_s = sg - sg.sum(axis=0)[None] / 3.0
    return loss, weight * g_s * s


# ---------------------------------------------------------------------------
# Eq. S1-S2: covisibility between keyframes.

def covisibility(visible):
    """visible: [V][n] bool.  Returns (iou [V][V], oc [V][V], counts [V]); a ratio whose
    denominator is zero is 0."""
    vis = np.asarray(visible, dtype=bool)
    V = vis.shape[0]
    counts = vis.sum(axis=1)
    iou = np.zeros((V, V))
    oc = np.zeros((V, V))
    for i in range(V):
        for j in range(V):
            inter = int((vis[i] & vis[j]).sum())
            union = int((vis[i] | vis[j]).sum())
            lo = min(counts[i], counts[j])
            iou[i, j] = inter / union if union else 0.0
            oc[i, j] = inter / lo if lo else 0.0
    return iou, oc, counts


def median_depth(depth):
    """Median of the positive entries (the lower middle element for an even count; 0 if
    there are none)."""
    d = np.sort(np.asarray(depth, dtype=np.float64).ravel())
    d = d[d > 0]
    if d.size == 0:
        return 0.0
    return float(d[(d.size - 1) // 2])
