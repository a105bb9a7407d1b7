"""GPU (HIP) vs FP64 oracle: RANSAC + PnP pose initialisation (Sec. 3.2.1, Eq. 6-9) through
the C ABI, on the same correspondences and the same caller-drawn samples."""
import numpy as np
import pytest

from paper_2507_03737_amd import scenes
from tests import gpu_util as U
from tests.test_oracle_tracking_pins import K, _problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CAM = scenes.Camera(960, 640, K[0], K[1], K[2], K[3])


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_03737_amd import binding
    binding.load()
    return binding


def _gpu(X, uv, samples, thr, iters=10, rounds=2, T_ak=None):
    from paper_2507_03737_amd.tracking import PnpConfig, pnp_ransac
    cfg = PnpConfig(n_hypotheses=len(samples), threshold=thr, iterations=iters, rounds=rounds)
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    uvd = torch.from_numpy(np.ascontiguousarray(uv, dtype=np.float32)).cuda()
    sd = torch.from_numpy(np.ascontiguousarray(samples, dtype=np.int32)).cuda()
    Tak = None if T_ak is None else torch.from_numpy(np.ascontiguousarray(T_ak, dtype=np.float32)).cuda()
    T, cnt, mask, scores, Tn = pnp_ransac(Xd, uvd, CAM, sd, cfg, T_ak=Tak)
    torch.cuda.synchronize()
    return (T.cpu().numpy(), int(cnt.item()), mask.cpu().numpy().astype(bool), scores.cpu().numpy(),
            None if Tn is None else Tn.cpu().numpy())


@pytest.mark.parametrize("case", ["exact_outliers", "noisy"])
def test_pnp_vs_oracle(lib, case):
    from oracle import tracking as TK
    U.log(f"[gpu] RANSAC + PnP ({case})")
    if case == "exact_outliers":
        X, uv, T_true, bad, samples = _problem(3000, 11, outliers=0.4)
        thr = 2.0
    else:
        X, uv, T_true, bad, samples = _problem(3000, 12, outliers=0.2, noise=0.7)
        thr = 3.0
    # Both sides see the float32 inputs the library receives.
    X32, uv32 = X.astype(np.float32).astype(np.float64), uv.astype(np.float32).astype(np.float64)
    ref = TK.pnp_ransac(X32, uv32, K, samples, thr=thr)
    T, cnt, mask, scores, _ = _gpu(X, uv, samples, thr)
    good = ref["gaps"] > 1e-6
    agree = (scores == ref["scores"])[good].mean()
    U.log(f"  best gpu {int(np.argmax(scores))} oracle {ref['best']}  inliers {cnt}/{int(ref['inliers'].sum())} "
          f"score agreement {agree:.4f}  |dT| {np.abs(T - ref['T']).max():.2e}  margin {ref['margin']:.1e}")
    assert agree >= 0.99
    assert int(np.argmax(scores)) == ref["best"]
    np.testing.assert_allclose(T, ref["T"], atol=1e-9)
    if ref["margin"] > 1e-9:
        assert np.array_equal(mask, ref["inliers"]) and cnt == int(ref["inliers"].sum())
    if case == "exact_outliers":
        np.testing.assert_allclose(T, T_true, atol=1e-6)   # float32 inputs


def test_pnp_invalid_samples_and_pose_composition(lib):
    from oracle import tracking as TK
    X, uv, T_true, bad, samples = _problem(500, 13, outliers=0.1)
    samples = samples[:64].copy()
    samples[3, 2] = -1
    samples[7, 5] = 500                                    # out of range
    T_ak = np.asarray(scenes.perturb_pose(np.concatenate([np.eye(3), np.zeros((3, 1))], 1).reshape(-1), 5.0, 2.0, 4),
                      np.float64)
    T, cnt, mask, scores, Tn = _gpu(X, uv, samples, 2.0, T_ak=T_ak)
    assert scores[3] == -1 and scores[7] == -1
    ref = TK.compose(T, T_ak.reshape(3, 4)).reshape(-1)
    np.testing.assert_allclose(Tn, ref.astype(np.float32), rtol=0, atol=2e-6)


def test_pnp_argument_errors(lib):
    from paper_2507_03737_amd.tracking import PnpConfig, pnp_ransac
    X = torch.zeros(3, 5, device="cuda")
    uv = torch.zeros(2, 5, device="cuda")
    s = torch.zeros(4, 6, dtype=torch.int32, device="cuda")
    with pytest.raises(lib.GspmError):                     # fewer than 6 correspondences
        pnp_ransac(X, uv, CAM, s, PnpConfig(n_hypotheses=4))
    X = torch.zeros(3, 10, device="cuda")
    uv = torch.zeros(2, 10, device="cuda")
    with pytest.raises(lib.GspmError):
        pnp_ransac(X, uv, CAM, s, PnpConfig(n_hypotheses=4, threshold=0.0))
