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
    for v, cam in enumerate(sc.cams):
        view = O.make_view(cam, sc.T_cw[v])
        pix = O.full_pixels(cam)
        r = O.render(po, view, S, pix)
        tr = O.trace(po, view, S, pix)
        amb = r["ambiguous"] != 0
        sure, loose = set(), set()
        for k in range(pix.shape[0]):
            gs = tr.frag_g[tr.offsets[k]:tr.offsets[k + 1]].tolist()
            (loose if amb[k] else sure).update(gs)
        got = set(np.flatnonzero(vis[v]).tolist())
        U.log(f"  view {v}: gpu {len(got)} oracle {len(sure)} (+{len(loose - sure)} on ambiguous pixels)")
        assert sure <= got
        assert len(got - sure - loose) <= max(2, len(got) // 200)
    ref_iou, ref_oc, ref_cnt = M.covisibility(vis)
    np.testing.assert_array_equal(iou.cpu().numpy(), ref_iou)
    np.testing.assert_array_equal(oc.cpu().numpy(), ref_oc)
    np.testing.assert_array_equal(cnt.cpu().numpy(), ref_cnt)
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
