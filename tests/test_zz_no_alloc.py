"""The allocation-free window loss (gspm_window_loss_noalloc) against gspm_window_loss.

Both run the same kernels on the same inputs; the allocation-free call keeps its per-wave
loss partials in the library's static device array instead of the context's scratch, so
the scale, the loss and both gradients must agree bit for bit.  Two calls in a row, the
second on a smaller window, show that the shared array keeps no state between calls that
matters.
"""
import ctypes

import numpy as np
import pytest

from paper_2507_03737_amd import scenes
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_03737_amd import binding
    binding.load()
    return binding


def _window(cams, seed):
    rng = np.random.default_rng(seed)
    P = sum(c.width * c.height for c in cams)
    f = lambda *shape: torch.from_numpy(rng.standard_normal(shape).astype(np.float32)).cuda()  # noqa: E731
    pm = f(3 * P) * 4.0
    prior = pm * 1.1 + f(3 * P) * 0.05
    return {"rgb": f(3 * P), "target": f(3 * P), "pm": pm, "prior": prior}


def _run(lib, cams, data, patch, alpha, noalloc, ctx=None):
    intr = lib.make_intrinsics(cams)
    T = torch.zeros(len(cams), 12, device="cuda")
    views = lib.make_views(intr, len(cams), T)
    P = sum(c.width * c.height for c in cams)
    n_patches = sum(-(-c.width // patch) * -(-c.height // patch) for c in cams)
    out = {"scale": torch.full((n_patches,), float("nan"), device="cuda"),
           "loss": torch.full((len(cams),), float("nan"), device="cuda"),
           "g_rgb": torch.full((3 * P,), float("nan"), device="cuda"),
           "g_pm": torch.full((3 * P,), float("nan"), device="cuda")}
    args = (data["rgb"], data["target"], data["pm"], data["prior"], patch, alpha, out["scale"], out["loss"],
            out["g_rgb"], out["g_pm"], lib.stream_handle())
    if noalloc:
        lib.window_loss_noalloc(views, *args)
    else:
        lib.window_loss(ctx, views, *args)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_noalloc_window_loss_matches_context_call(lib):
    """Two calls in a row, the second on a smaller window, each checked element by element
    against the context-scratch entry point on the same inputs."""
    ctx = lib.Context()
    big = [scenes.Camera(960, 640, 572.0, 572.0, 480.0, 320.0), scenes.Camera(1216, 352, 724.6, 724.6, 608.0, 176.0),
           scenes.Camera(640, 480, 381.0, 381.0, 320.0, 240.0)]
    small = [scenes.Camera(157, 93, 100.0, 100.0, 78.5, 46.5)]
    for tag, cams, patch, seed in (("window of 3 views", big, 8, 1), ("small ragged view", small, 10, 2)):
        U.log(f"[gpu] noalloc window loss: {tag}, patch {patch}")
        data = _window(cams, seed)
        ref = _run(lib, cams, data, patch, 0.98, noalloc=False, ctx=ctx)
        got = _run(lib, cams, data, patch, 0.98, noalloc=True)
        for k in ref:
            assert np.all(np.isfinite(got[k])), k
            assert np.array_equal(got[k], ref[k]), f"{tag}: {k} differs"
    ctx.close()


def test_noalloc_window_loss_rejects_oversize(lib):
    """A window that needs more partial slots than the static array holds is refused
    before any launch."""
    cams = [scenes.Camera(4096, 4096, 2000.0, 2000.0, 2048.0, 2048.0)] * 8
    intr = lib.make_intrinsics(cams)
    views = lib.make_views(intr, len(cams), torch.zeros(len(cams), 12, device="cuda"))
    st = lib.load().gspm_window_loss_noalloc(ctypes.byref(views), 1, 1, 1, 1, 1, ctypes.c_float(0.5), 1, 1, 1, 1,
                                             None)
    assert st == lib.GSPM_ERR_INVALID_ARG and "partials" in lib.last_error()
