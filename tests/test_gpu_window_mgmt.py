"""GPU (HIP) vs FP64 oracle: the isotropic regulariser (Eq. 16), keyframe covisibility
(supplementary Eq. S1-S2) from the forward's contributing-record marks, and the median
rendered depth, through the C ABI."""
import numpy as np
import pytest

from paper_2507_03737_amd import scenes
from tests import gpu_util as U
from tests.test_gpu_parity import _oracle_settings

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_03737_amd import binding
    binding.load()
    return binding


def test_iso_loss_vs_oracle(lib):
    from oracle import mapping as M
    from paper_2507_03737_amd.render import Rasterizer, Window
    U.log("[gpu] isotropic regulariser")
    sc = scenes.make_scene("c1")
    ls = sc.log_scales.copy()
    ls[:, :1000] = ls[0, :1000][None]                  # exactly isotropic Gaussians
    sc.log_scales = ls
    params, T = U.to_dev(sc, torch)
    rast = Rasterizer(Window(sc.cams, T), sc.n, lib.RasterConfig())
    g0 = torch.randn(3, sc.n, device="cuda")
    grad = g0.clone()
    loss = torch.empty(1, device="cuda")
    rast.iso_loss_into(params, 10.0, loss, grad)
    torch.cuda.synchronize()
    ref_loss, ref_g = M.iso_loss(ls, weight=10.0)
    assert abs(float(loss.item()) - ref_loss) <= 1e-6 * ref_loss
    got = (grad - g0).cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, ref_g, rtol=1e-6, atol=1e-6 * np.abs(ref_g).max())
    assert not got[:, :1000].any()


def test_covisibility_vs_oracle(lib, oracle):
    """Visible sets (Gaussians contributing to at least one pixel of a view) equal the
    oracle's, except for Gaussians that are candidates of a pixel the oracle flags as
    ambiguous, where a float32 decision may legitimately differ.  IOU and OC (Eq. S1-S2)
    computed from the oracle's sets bound the GPU's: changing k set members moves an
    intersection and a union by at most k each."""
    from oracle import mapping as M
    from paper_2507_03737_amd.render import Rasterizer, Window
    from tests.test_gpu_window import _window_scene
    U.log("[gpu] covisibility")
    O = oracle
    sc = _window_scene(seed=16)
    params, T = U.to_dev(sc, torch)
    win = Window(sc.cams, T)
    rast = Rasterizer(win, sc.n, lib.RasterConfig(mark_visible=1))
    out, fs = rast.forward(params)
    iou, oc, cnt = rast.covisibility(fs)
    torch.cuda.synchronize()
    V = len(sc.cams)
    lay = U.frame_layout(0, 0, sc.n * V)
    vis = fs.cpu().numpy()[lay["visible"]:lay["visible"] + sc.n * V].reshape(V, sc.n) != 0
    S = _oracle_settings(O, rast.cfg)
    po = O.Params.from_scene(sc)
    ref_vis = np.zeros_like(vis)
    unsure = np.zeros_like(vis)
    for v, cam in enumerate(sc.cams):
        view = O.make_view(cam, sc.T_cw[v])
        pix = O.full_pixels(cam)
        r = O.render(po, view, S, pix)
        tr = O.trace(po, view, S, pix)
        ref_vis[v, np.unique(tr.frag_g)] = True
        pa = O.proj_numpy(O.project(po, view, S))
        cr = pa["crect"]
        for i, j in pix[r["ambiguous"] != 0]:
            unsure[v] |= (pa["cand"] == 1) & (cr[:, 0] <= i) & (i <= cr[:, 1]) & (cr[:, 2] <= j) & (j <= cr[:, 3])
        diff = vis[v] != ref_vis[v]
        U.log(f"  view {v}: gpu {int(vis[v].sum())} oracle {int(ref_vis[v].sum())}, differing {int(diff.sum())}, "
              f"candidates of flagged pixels {int(unsure[v].sum())}")
        assert not (diff & ~unsure[v]).any(), f"view {v}: sets differ off ambiguous pixels"
    got_iou, got_oc, got_cnt = iou.cpu().numpy(), oc.cpu().numpy(), cnt.cpu().numpy()
    # The GPU's IOU/OC are those of its own sets, exactly ...
    g_iou, g_oc, g_cnt = M.covisibility(vis)
    np.testing.assert_array_equal(got_iou, g_iou)
    np.testing.assert_array_equal(got_oc, g_oc)
    np.testing.assert_array_equal(got_cnt, g_cnt)
    # ... and within the bound of the oracle's.
    r_iou, r_oc, _ = M.covisibility(ref_vis)
    for i in range(V):
        for j in range(V):
            k = int((unsure[i] | unsure[j]).sum())
            union = int((ref_vis[i] | ref_vis[j]).sum())
            small = int(min(ref_vis[i].sum(), ref_vis[j].sum()))
            assert abs(got_iou[i, j] - r_iou[i, j]) <= 2 * k / max(1, union - k) + 1e-12
            assert abs(got_oc[i, j] - r_oc[i, j]) <= 2 * k / max(1, small - k) + 1e-12
    # Without marking, the call reports it instead of returning stale sets.
    rast2 = Rasterizer(win, sc.n, lib.RasterConfig())
    _, fs2 = rast2.forward(params)
    iou2, _, cnt2 = rast2.covisibility(fs2)
    assert torch.isnan(iou2).all() and (cnt2 == -1).all()


def test_median_depth_vs_oracle(lib):
    from oracle import mapping as M
    from paper_2507_03737_amd.render import Rasterizer, Window
    U.log("[gpu] median depth")
    cams = [scenes.Camera(960, 640, 572.0, 572.0, 480.0, 320.0), scenes.Camera(157, 93, 110.0, 110.0, 78.5, 46.5),
            scenes.Camera(64, 48, 50.0, 50.0, 32.0, 24.0), scenes.Camera(33, 17, 30.0, 30.0, 16.5, 8.5)]
    rng = np.random.default_rng(3)
    depths = []
    for k, c in enumerate(cams):
        d = scenes.street_pointmap(c, 30 + k)[2].copy()
        d[rng.random(d.shape) < 0.3] = 0.0                 # pixels without Gaussians
        depths.append(d)
    depths[2][:] = 0.0                                     # an empty view
    depths[3].reshape(-1)[:] = np.float32(7.25)             # all equal
    T = torch.zeros(len(cams), 12, device="cuda")
    rast = Rasterizer(Window(cams, T), 1, lib.RasterConfig())
    d = torch.from_numpy(np.concatenate([x.reshape(-1) for x in depths])).cuda()
    med = rast.median_depth(d).cpu().numpy()
    for k in range(len(cams)):
        assert med[k] == np.float32(M.median_depth(depths[k])), k
