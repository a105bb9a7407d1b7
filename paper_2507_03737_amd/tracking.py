"""Pose initialisation of a new frame from the adjacent keyframe (Sec. 3.2.1, Eq. 6-9).

The 3D side of the 2D-3D correspondences comes from the keyframe's rendered pointmap
(camera frame), so the relative pose carries the map's own scale.  ``pnp_ransac`` runs
the library's RANSAC + PnP (six-point linear hypotheses, scoring, Gauss-Newton refinement
on the inliers) and returns T_rel and, given the keyframe pose, T_n = T_rel T_ak (Eq. 9).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import binding as B

__all__ = ["PnpConfig", "pnp_ransac", "draw_samples"]


@dataclass
class PnpConfig:
    n_hypotheses: int = 1024
    threshold: float = 2.0   # pixels
    iterations: int = 10
    rounds: int = 2

    def c(self) -> B.PnpParams:
        return B.PnpParams(self.n_hypotheses, self.threshold, self.iterations, self.rounds)


def draw_samples(n: int, n_hypotheses: int, generator: torch.Generator | None = None, device="cuda"):
    """[H][6] int32 sample indices drawn uniformly (with replacement) on the device."""
    return torch.randint(0, n, (n_hypotheses, 6), dtype=torch.int32, device=device, generator=generator)


def pnp_ransac(X: torch.Tensor, uv: torch.Tensor, cam, samples: torch.Tensor, cfg: PnpConfig | None = None,
               T_ak: torch.Tensor | None = None, ctx: B.Context | None = None, stream=None):
    """X [3][n], uv [2][n] (float32, device).  Returns (T_rel [3][4] float64, inlier count [1],
    inlier mask [n], scores [H], T_n [12] float32 = T_rel T_ak or None without T_ak)."""
    cfg = cfg or PnpConfig()
    ctx = ctx or B.Context()
    if samples.shape != (cfg.n_hypotheses, 6) or samples.dtype != torch.int32:
        raise ValueError("samples must be int32 [n_hypotheses][6]")
    dev = X.device
    T = torch.empty(12, dtype=torch.float64, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    mask = torch.empty(X.shape[-1], dtype=torch.uint8, device=dev)
    scores = torch.empty(cfg.n_hypotheses, dtype=torch.int32, device=dev)
    T_n = torch.empty(12, dtype=torch.float32, device=dev) if T_ak is not None else None
    K = B.Intrinsics(int(cam.width), int(cam.height), float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy))
    B.pnp_ransac(ctx, X.contiguous(), uv.contiguous(), K, samples.contiguous(), cfg.c(), T, cnt, mask, scores,
                 None if T_ak is None else T_ak.contiguous(), T_n, B.stream_handle(stream))
    return T.view(3, 4), cnt, mask, scores, T_n
