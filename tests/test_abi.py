"""The C ABI library loads, exports every entry point declared in include/gspm.h and
rejects bad arguments on the host, before any HIP call (runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2507_03737_amd import binding as B
from paper_2507_03737_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gspm.h")).read()
    return sorted(set(re.findall(r"GSPM_API\s+[\w\s\*]+?\b(gspm_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(B.LIB_PATH):
        from paper_2507_03737_amd import build
        build.build(verbose=False)
    return B.load()


def test_every_declared_symbol_is_exported(L):
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(B.EXPORTS)
    assert B.version().startswith("gspm")


def _views(intr, n_views=1, T=1):
    return B.Views(n_views, ctypes.cast(intr, ctypes.POINTER(B.Intrinsics)), T)


def test_frame_state_bytes_validation(L):
    intr = B.make_intrinsics([scenes.Camera(160, 120, 128.0, 128.0, 80.0, 60.0)])
    v = _views(intr)
    nb = B.frame_state_bytes(v, 2000, 1000, 16)
    assert nb > 2000 * 64 + 1000 * 4
    assert L.gspm_frame_state_bytes(ctypes.byref(v), 10, 10, 12) == -1
    assert "tile" in B.last_error()
    bad = B.make_intrinsics([scenes.Camera(0, 120, 128.0, 128.0, 80.0, 60.0)])
    assert L.gspm_frame_state_bytes(ctypes.byref(_views(bad)), 10, 10, 16) == -1
    assert "size" in B.last_error()
    assert L.gspm_frame_state_bytes(ctypes.byref(_views(intr, 0)), 10, 10, 16) == -1
    assert L.gspm_frame_state_bytes(ctypes.byref(_views(intr, 33)), 10, 10, 16) == -1


def test_forward_argument_errors_before_any_launch(L):
    ctx = ctypes.c_void_p()
    assert L.gspm_create(ctypes.byref(ctx)) == B.GSPM_OK
    intr = B.make_intrinsics([scenes.Camera(160, 120, 128.0, 128.0, 80.0, 60.0)])
    v = _views(intr)
    g = B.Gaussians(1, 1, 1, 1, 1, 10)
    img = B.Images(1, 1, 1, 1)
    cfg = B.RasterConfig().c()

    def fwd(ctx_=ctx, g_=g, v_=v, s_=cfg, o_=img, fs=1, nbytes=1 << 30):
        return L.gspm_render_forward(ctx_, ctypes.byref(g_) if g_ is not None else None, ctypes.byref(v_),
                                     ctypes.byref(s_), ctypes.byref(o_), fs, nbytes, None)

    assert fwd(ctx_=None) == B.GSPM_ERR_INVALID_ARG
    assert fwd(g_=None) == B.GSPM_ERR_INVALID_ARG
    assert fwd(g_=B.Gaussians(0, 1, 1, 1, 1, 10)) == B.GSPM_ERR_INVALID_ARG
    assert fwd(g_=B.Gaussians(1, 1, 1, 1, 1, -1)) == B.GSPM_ERR_INVALID_ARG
    assert fwd(o_=B.Images(1, 0, 1, 1)) == B.GSPM_ERR_INVALID_ARG
    assert fwd(fs=None) == B.GSPM_ERR_INVALID_ARG
    assert fwd(nbytes=16) == B.GSPM_ERR_INVALID_ARG and "frame_state_bytes" in B.last_error()
    for field, val in (("tile", 12), ("pixels_per_lane", 3), ("sort_digit_bits", 9), ("pointmap_frame", 3), ("alpha_min", 0.0),
                       ("alpha_max", 1.0), ("t_min", 0.0), ("near_z", -1.0), ("eps2d", -0.1), ("jac_clamp", 0.0)):
        s = B.RasterConfig().c()
        setattr(s, field, val)
        assert fwd(s_=s) == B.GSPM_ERR_INVALID_ARG, field
    s = B.RasterConfig().c()
    s.bg[1] = float("nan")
    assert fwd(s_=s) == B.GSPM_ERR_INVALID_ARG
    L.gspm_destroy(ctx)


def test_backward_and_loss_argument_errors(L):
    ctx = ctypes.c_void_p()
    assert L.gspm_create(ctypes.byref(ctx)) == B.GSPM_OK
    intr = B.make_intrinsics([scenes.Camera(16, 16, 10.0, 10.0, 8.0, 8.0)])
    v = _views(intr)
    g = B.Gaussians(1, 1, 1, 1, 1, 3)
    cfg = B.RasterConfig().c()
    f = B.Images(1, 1, 1, 1)
    u = B.Images(0, 0, 0, 0)
    assert L.gspm_render_backward(ctx, ctypes.byref(g), ctypes.byref(v), ctypes.byref(cfg), ctypes.byref(f),
                                  ctypes.byref(u), 1, None, None, None) == B.GSPM_ERR_INVALID_ARG
    assert L.gspm_pose_backward(ctx, ctypes.byref(g), ctypes.byref(v), ctypes.byref(cfg), ctypes.byref(f),
                                ctypes.byref(u), 1, None, None) == B.GSPM_ERR_INVALID_ARG
    assert L.gspm_render_backward(ctx, ctypes.byref(g), ctypes.byref(v), ctypes.byref(cfg),
                                  ctypes.byref(B.Images(1, 0, 1, 1)), ctypes.byref(u), 1, None, 1,
                                  None) == B.GSPM_ERR_INVALID_ARG
    assert L.gspm_patch_scale_align(ctypes.byref(v), 1, 1, None, 0, 1, None, None) == B.GSPM_ERR_INVALID_ARG
    assert L.gspm_patch_scale_align(ctypes.byref(v), None, 1, None, 8, 1, None, None) == B.GSPM_ERR_INVALID_ARG
    assert L.gspm_window_loss(ctx, ctypes.byref(v), 1, 1, 1, 1, 8, ctypes.c_float(1.5), 1, 1, 1, 1,
                              None) == B.GSPM_ERR_INVALID_ARG
    assert L.gspm_window_loss(None, ctypes.byref(v), 1, 1, 1, 1, 8, ctypes.c_float(0.5), 1, 1, 1, 1,
                              None) == B.GSPM_ERR_INVALID_ARG
    assert L.gspm_patch_scale_align(ctypes.byref(v), 1, 1, None, 65, 1, None, None) == B.GSPM_ERR_INVALID_ARG
    assert L.gspm_pose_retract(0, 1, 1, None) == B.GSPM_ERR_INVALID_ARG
    L.gspm_destroy(ctx)


def test_product_path_has_no_oracle_or_cpu_fallback():
    """The package never imports the oracle, and the binding raises when the library is absent."""
    pkg = os.path.join(ROOT, "paper_2507_03737_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", txt, re.M), f
                assert "liboracle" not in txt and "gs_oracle" not in txt, f
    with pytest.raises(B.GspmError):
        saved = B._lib
        try:
            B._lib = None
            B.load(os.path.join(ROOT, "does-not-exist.so"))
        finally:
            B._lib = saved


def test_sort_limits_and_noalloc_size_checked_on_host(L):
    """Counts the radix sorts cannot take (2^30 keys and more) and windows beyond the
    allocation-free loss's static array are refused on the host, before any HIP call."""
    ctx = ctypes.c_void_p()
    assert L.gspm_create(ctypes.byref(ctx)) == B.GSPM_OK
    assert L.gspm_reserve(ctx, 1 << 30, 10, 10) == B.GSPM_ERR_INVALID_ARG and "2^30" in B.last_error()
    assert L.gspm_reserve(ctx, 10, 1 << 30, 10) == B.GSPM_ERR_INVALID_ARG
    intr = B.make_intrinsics([scenes.Camera(160, 120, 128.0, 128.0, 80.0, 60.0)] * 2)
    v = _views(intr, 2)
    g = B.Gaussians(1, 1, 1, 1, 1, 1 << 29)
    cfg = B.RasterConfig().c()
    assert L.gspm_render_forward(ctx, ctypes.byref(g), ctypes.byref(v), ctypes.byref(cfg),
                                 ctypes.byref(B.Images(1, 1, 1, 1)), 1, 1 << 40, None) == B.GSPM_ERR_INVALID_ARG
    assert "2^30" in B.last_error()
    big = B.make_intrinsics([scenes.Camera(4096, 4096, 2000.0, 2000.0, 2048.0, 2048.0)] * 8)
    st = L.gspm_window_loss_noalloc(ctypes.byref(_views(big, 8)), 1, 1, 1, 1, 1, ctypes.c_float(0.5), 1, 1, 1, 1,
                                    None)
    assert st == B.GSPM_ERR_INVALID_ARG and "partials" in B.last_error()
    assert L.gspm_window_loss_noalloc(ctypes.byref(v), 1, 1, None, 1, 8, ctypes.c_float(0.5), 1, 1, 1, 1,
                                      None) == B.GSPM_ERR_INVALID_ARG
    assert L.gspm_window_loss_noalloc(ctypes.byref(v), 1, 1, 1, 1, 8, ctypes.c_float(2.0), 1, 1, 1, 1,
                                      None) == B.GSPM_ERR_INVALID_ARG
    L.gspm_destroy(ctx)
