"""The wave culling's geometry (host-side check of the argument the kernel relies on).

A record's exponent over the image plane is a concave quadratic with its maximum at the
mean (Sec. 3.1, the tile-based rasterization of the projected Gaussians).  The forward's
per-wave rectangle test evaluates it on two segments only: the column x = clamp(u, x0, x1)
over [y0, y1] and the row y = clamp(v, y0, y1) over [x0, x1].  These tests check, in FP64
and by brute force over a fine grid, that the maximum over the whole rectangle is the
larger of the two segment maxima, for random conics (thin and rotated ones included),
means inside, beside and diagonal to the rectangle.
"""
import numpy as np


def _segment_max(P, Q, R, d, lo, hi):
    """Largest P d^2 + Q d t + R t^2 (R < 0) over t in [lo, hi], for fixed d."""
    t = np.clip(-0.5 * Q * d / R, lo, hi)
    return P * d * d + Q * d * t + R * t * t


def _two_segment_max(A, B, C, u, v, x0, x1, y0, y1):
    ax, bx, ay, by = x0 - u, x1 - u, y0 - v, y1 - v
    cx = np.clip(0.0, ax, bx)
    cy = np.clip(0.0, ay, by)
    return max(_segment_max(A, B, C, cx, ay, by), _segment_max(C, B, A, cy, ax, bx))


def _grid_max(A, B, C, u, v, x0, x1, y0, y1, n=161):
    xs = np.linspace(x0, x1, n)
    ys = np.linspace(y0, y1, n)
    dx = xs[None, :] - u
    dy = ys[:, None] - v
    return float(np.max(A * dx * dx + B * dx * dy + C * dy * dy))


def _boundary_max(A, B, C, u, v, x0, x1, y0, y1):
    """The maximum over the rectangle from its definition: 0 if the mean lies inside,
    else the largest of the four edge maxima (a concave function's maximum over a convex
    polygon that does not hold its peak lies on the boundary)."""
    ax, bx, ay, by = x0 - u, x1 - u, y0 - v, y1 - v
    if ax <= 0 <= bx and ay <= 0 <= by:
        return 0.0
    return max(_segment_max(A, B, C, ax, ay, by), _segment_max(A, B, C, bx, ay, by),
               _segment_max(C, B, A, ay, ax, bx), _segment_max(C, B, A, by, ax, bx))


def _random_conic(rng):
    # Factored form e = -((a dx + b dy)^2 + (c dy)^2), as the records store it.
    a = np.exp(rng.uniform(-3.0, 1.0))
    c = np.exp(rng.uniform(-3.0, 1.0))
    b = rng.uniform(-2.0, 2.0) * max(a, c)
    return -a * a, -2.0 * a * b, -(b * b + c * c)


def test_two_segments_hold_the_rectangle_maximum():
    rng = np.random.default_rng(20250703)
    for _ in range(400):
        A, B, C = _random_conic(rng)
        x0, y0 = rng.uniform(-4, 4, size=2)
        x1, y1 = x0 + rng.uniform(0, 7), y0 + rng.uniform(0, 7)
        u, v = rng.uniform(-25, 25, size=2)
        two = _two_segment_max(A, B, C, u, v, x0, x1, y0, y1)
        full = _boundary_max(A, B, C, u, v, x0, x1, y0, y1)
        grid = _grid_max(A, B, C, u, v, x0, x1, y0, y1)
        assert abs(two - full) <= 1e-12 * (1.0 + abs(full))
        # Brute force: no grid point of the rectangle lies above it.
        assert grid <= full + 1e-12 * (1.0 + abs(full))


def test_mean_inside_gives_zero():
    rng = np.random.default_rng(7)
    for _ in range(50):
        A, B, C = _random_conic(rng)
        x0, y0 = rng.uniform(-4, 4, size=2)
        x1, y1 = x0 + rng.uniform(0.5, 7), y0 + rng.uniform(0.5, 7)
        u, v = rng.uniform(x0, x1), rng.uniform(y0, y1)
        assert _two_segment_max(A, B, C, u, v, x0, x1, y0, y1) == 0.0


def test_far_edges_alone_would_miss_the_maximum():
    """A thin rotated conic whose mean lies left of the rectangle reaches it highest on the
    facing (left) edge, not on the far one: the row through the clamped mean and the facing
    column are what the test evaluates, and they find it."""
    a, b, c = 1.0, -3.0, 0.05
    A, B, C = -a * a, -2.0 * a * b, -(b * b + c * c)
    x0, x1, y0, y1 = 0.0, 7.0, 0.0, 7.0
    u, v = -2.0, 3.0
    grid = _grid_max(A, B, C, u, v, x0, x1, y0, y1, 701)
    far = _segment_max(A, B, C, x1 - u, y0 - v, y1 - v)
    two = _two_segment_max(A, B, C, u, v, x0, x1, y0, y1)
    assert far < grid - 1e-3
    assert abs(two - grid) <= 1e-4 * (1.0 + abs(grid))
