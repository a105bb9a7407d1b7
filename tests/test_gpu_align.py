"""GPU (HIP) vs FP64 oracle: patch-based scale alignment (supplementary Alg. 1) and
pointmap replacement (Eq. 14), through the C ABI, on a window of uneven views with masks,
outlier patches and pixels, a view without candidates and a fully masked view."""
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


def _window():
    cams = [scenes.Camera(1216, 352, 724.6, 724.6, 608.0, 176.0), scenes.Camera(157, 93, 110.0, 110.0, 78.5, 46.5),
            scenes.Camera(160, 120, 128.0, 128.0, 80.0, 60.0), scenes.Camera(64, 48, 50.0, 50.0, 32.0, 24.0)]
    scales = [1.15, 0.87, 2.0, 1.0]
    Xr = [scenes.street_pointmap(c, 10 + k) for k, c in enumerate(cams)]
    Xp = [scenes.noisy_prior(x, s, 20 + k) for k, (x, s) in enumerate(zip(Xr, scales))]
    # View 2: every patch at twice the scale, so no patch is ever a candidate.
    Xp[2] = scenes.noisy_prior(Xr[2], 2.0, 22, outlier_patches=0.0, outlier_pixels=0.0)
    rng = np.random.default_rng(5)
    masks = [np.ones((c.height, c.width), np.float32) for c in cams]
    masks[1] = (rng.random((93, 157)) > 0.2).astype(np.float32)
    masks[3][:] = 0.0
    return cams, Xr, Xp, masks


def _run(lib, cams, Xr, Xp, masks, cfg):
    from paper_2507_03737_amd.render import Rasterizer, Window, align_results
    T = torch.zeros(len(cams), 12, device="cuda")
    T[:, 0] = T[:, 5] = T[:, 10] = 1.0
    rast = Rasterizer(Window(cams, T), 1, lib.RasterConfig())
    cat = lambda arrs: torch.from_numpy(np.concatenate([a.reshape(-1) for a in arrs])).cuda()  # noqa: E731
    xr, xp, m = cat(Xr), cat(Xp), cat(masks)
    res = rast.new_align_result()
    rast.align_scale_into(xr, xp, res, mask=m, cfg=cfg)
    hat = torch.empty_like(xr)
    rep = torch.empty(len(cams), dtype=torch.int32, device="cuda")
    rast.replace_pointmap_into(xr, xp, res, hat, rep, eps_m=cfg.eps_m)
    torch.cuda.synchronize()
    return align_results(res), hat.cpu().numpy(), rep.cpu().numpy()


@pytest.mark.parametrize("patch", [10, 7, 64])
def test_align_and_replace_vs_oracle(lib, patch):
    from oracle import mapping as M
    U.log(f"[gpu] scale alignment + replacement, patch {patch}")
    cams, Xr, Xp, masks = _window()
    cfg = lib.AlignConfig(patch=patch)
    got, hat, rep = _run(lib, cams, Xr, Xp, masks, cfg)
    off = 0
    for v, cam in enumerate(cams):
        r = M.align_scale(Xr[v], Xp[v], P=patch, delta_mu=cfg.delta_mu, delta_sigma=cfg.delta_sigma, eps_r=cfg.eps_r,
                          max_iter=cfg.max_iter, tau=cfg.tau, mask=masks[v])
        g = got[v]
        U.log(f"  view {v}: scale gpu {g['scale']:.12f} oracle {r['scale']:.12f}  cp {g['cp']}/{r['cp']} "
              f"valid {g['n_valid']}  margin {r['margin']:.2e}")
        assert g["n_valid"] == r["n_valid"]
        assert abs(g["scale"] - r["scale"]) <= 1e-9 * abs(r["scale"])
        if r["margin"] > 1e-9:
            assert g["cp"] == r["cp"] and bool(g["insufficient"]) == bool(r["insufficient"])
        ref, replaced, margin = M.replace_pointmap(Xr[v], Xp[v], g["scale"], cfg.eps_m)
        n3 = 3 * cam.height * cam.width
        h = hat[off:off + n3].reshape(3, cam.height, cam.width)
        ref32 = ref.astype(np.float32)
        ulp = np.spacing(np.abs(ref32)).astype(np.float64)
        assert (np.abs(h.astype(np.float64) - ref32.astype(np.float64)) <= ulp).all(), f"view {v}"
        if margin > 1e-9:
            assert rep[v] == int(replaced.sum())
        off += n3
    assert got[2]["scale"] == 1.0 and got[2]["cp"] == 0 and got[2]["insufficient"] == 1   # no candidates
    assert got[3]["n_valid"] == 0 and got[3]["scale"] == 1.0                              # fully masked


def test_align_argument_errors(lib):
    from paper_2507_03737_amd.render import Rasterizer, Window
    cams, Xr, Xp, masks = _window()
    T = torch.zeros(1, 12, device="cuda")
    rast = Rasterizer(Window(cams[:1], T), 1, lib.RasterConfig())
    x = torch.zeros(3 * cams[0].width * cams[0].height, device="cuda")
    res = rast.new_align_result()
    for bad in (lib.AlignConfig(patch=1), lib.AlignConfig(patch=65), lib.AlignConfig(max_iter=0),
                lib.AlignConfig(eps_r=0.0)):
        with pytest.raises(lib.GspmError):
            rast.align_scale_into(x, x, res, cfg=bad)
    rep = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(lib.GspmError):
        rast.replace_pointmap_into(x, x, res, x, rep)   # output aliases the input
