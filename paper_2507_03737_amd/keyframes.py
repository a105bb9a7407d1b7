"""Keyframe window management (supplementary keyframe-management section, Eq. S1-S2).

Host-side policy over quantities the library computes on the GPU: the covisibility IOU
and overlap coefficient of the visible Gaussian sets (``Rasterizer.covisibility``) and the
median rendered depth of a frame (``Rasterizer.median_depth``).  The paper's values are
k_I = 0.9, k_d = 0.08, k_o = 0.3 and a window of 8 keyframes.

Reading of the rules:
* a frame i becomes a keyframe when its covisibility with the latest keyframe j is low,
  IOU(i, j) < k_I, or when it has moved far relative to its own scene depth,
  d_ij > k_d * median_depth_i (d_ij the distance between the camera centres);
* when keyframe i' joins the window, every keyframe l with OC(i', l) < k_o leaves it;
  if the window is still larger than its maximum size, the keyframe with the lowest OC
  relative to i' leaves (repeatedly), and i' itself always stays.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Tuple

import numpy as np

__all__ = ["KeyframePolicy", "KeyframeWindow", "camera_distance"]


def camera_distance(T_a, T_b) -> float:
    """Distance between the camera centres of two world->camera poses (3x4 row-major)."""
    def centre(T):
        M = np.asarray(T, dtype=np.float64).reshape(3, 4)
        return -M[:, :3].T @ M[:, 3]
    return float(np.linalg.norm(centre(T_a) - centre(T_b)))


@dataclass
class KeyframePolicy:
    k_I: float = 0.9
    k_d: float = 0.08
    k_o: float = 0.3
    size: int = 8

    def is_keyframe(self, iou_with_latest: float, distance: float, median_depth: float) -> bool:
        return iou_with_latest < self.k_I or distance > self.k_d * median_depth


@dataclass
class KeyframeWindow:
    policy: KeyframePolicy = field(default_factory=KeyframePolicy)
    frames: List[int] = field(default_factory=list)

    def add(self, kf: int, oc_with_new: Dict[int, float]) -> Tuple[List[int], List[int]]:
        """Insert keyframe ``kf`` given OC(kf, l) for the keyframes l in the window.

        Returns (window after the update, keyframes removed)."""
        missing = [l for l in self.frames if l not in oc_with_new]
        if missing:
            raise ValueError(f"OC missing for keyframes {missing}")
        removed = [l for l in self.frames if oc_with_new[l] < self.policy.k_o]
        keep = [l for l in self.frames if oc_with_new[l] >= self.policy.k_o]
        while len(keep) + 1 > self.policy.size:
            worst = min(keep, key=lambda l: (oc_with_new[l], l))
            keep.remove(worst)
            removed.append(worst)
        self.frames = keep + [kf]
        return list(self.frames), removed
