"""Full-size parity in the benchmark's launch configurations: the c3 mapping window (1M
Gaussians, 8 views of uneven size, 16x16 tiles, 1 pixel per lane) and the c4 window (3M
Gaussians, 16 views of 1920x1080, 32x32 tiles, 2 pixels per lane), checked against the
oracle on sampled crops of every view (forward) and with upstream gradients confined to
those crops (backward to every parameter and every pose)."""
import numpy as np
import pytest

from paper_2507_03737_amd import scenes
from tests import gpu_util as U
from tests.test_gpu_parity import (_check_view_forward, _gpu_backward, _oracle_backward, _render_gpu,
                                   _upstream)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_03737_amd import binding
    binding.load()
    return binding


@pytest.mark.parametrize("name,tile,ppl,crop", [("c3", 16, 1, 16), ("c4", 32, 2, 8)])
def test_full_window_on_crops(lib, oracle, name, tile, ppl, crop):
    U.log(f"[gpu] {name} full size, tile {tile} ppl {ppl}, {crop}x{crop} crop per view")
    O = oracle
    sc = scenes.make_scene(name)
    cfg = lib.RasterConfig(pointmap_frame=1, tile=tile, pixels_per_lane=ppl)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    pix_sets, oks = [], []
    for v, cam in enumerate(sc.cams):
        boxes = U.crops(cam, crop, 1, seed=100 + v)
        pix = np.concatenate([O.crop_pixels(*b) for b in boxes])
        ref = _check_view_forward(O, sc, v, out, rast.win.pix_off[v], cfg, pixels=pix, tag=f"{name} v{v}")
        ok = np.zeros((cam.height, cam.width), bool)
        ok[pix[:, 1], pix[:, 0]] = ref["ambiguous"] == 0
        pix_sets.append(pix)
        oks.append(ok)
    ups = _upstream(sc, 9, oks)
    g = _gpu_backward(lib, rast, params, out, fs, ups)
    r = _oracle_backward(O, sc, cfg, ups, pixel_sets=pix_sets)
    for k in ("means", "log_scales", "quats", "opacity_logit", "rgb"):
        U.log(f"  {k}: rel {U.check_grad(name + ' ' + k, g[k], r[k]):.2e}")
    for v in range(len(sc.cams)):
        U.check_grad(f"{name} pose v{v}", g["pose"][v], r["pose"][v], frac=1.0)
