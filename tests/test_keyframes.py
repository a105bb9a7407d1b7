"""Host-side keyframe window policy (supplementary keyframe management)."""
import numpy as np
import pytest

from paper_2507_03737_amd.keyframes import KeyframePolicy, KeyframeWindow, camera_distance


def test_keyframe_rule():
    p = KeyframePolicy()
    assert p.is_keyframe(0.85, 0.0, 20.0)            # low covisibility
    assert not p.is_keyframe(0.95, 1.5, 20.0)        # 1.5 m < 0.08 * 20 m
    assert p.is_keyframe(0.95, 1.7, 20.0)            # moved beyond 8% of the median depth


def test_window_drops_low_overlap_and_caps_size():
    w = KeyframeWindow(KeyframePolicy(size=3))
    assert w.add(0, {}) == ([0], [])
    assert w.add(1, {0: 0.8}) == ([0, 1], [])
    assert w.add(2, {0: 0.5, 1: 0.9}) == ([0, 1, 2], [])
    # Window full: the lowest OC relative to the new keyframe leaves.
    frames, removed = w.add(3, {0: 0.4, 1: 0.6, 2: 0.95})
    assert frames == [1, 2, 3] and removed == [0]
    # OC below k_o = 0.3 removes regardless of size.
    frames, removed = w.add(4, {1: 0.1, 2: 0.5, 3: 0.7})
    assert frames == [2, 3, 4] and removed == [1]
    with pytest.raises(ValueError):
        w.add(5, {2: 0.5})


def test_camera_distance():
    R = np.eye(3)
    Ta = np.concatenate([R, [[0.0], [0.0], [0.0]]], axis=1)
    Tb = np.concatenate([R, [[0.0], [0.0], [-2.0]]], axis=1)   # centre at z = +2
    assert camera_distance(Ta, Tb) == pytest.approx(2.0)
