"""GPU tests of the tracking path (c2: 500k Gaussians, one 960x640 view): the pose-only
backward against the oracle and FP64 finite differences, and a 50-iteration pose loop."""
import dataclasses
import math

import numpy as np
import pytest

from paper_2507_03737_amd import scenes
from tests import gpu_util as U
from tests.test_gpu_parity import _check_view_forward, _oracle_settings, _upstream

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_03737_amd import binding
    binding.load()
    return binding


@pytest.fixture(scope="module")
def c2():
    return scenes.make_scene("c2")


def _pose_error(T12, T_true12):
    """Rotation angle (rad) and translation distance (m) of T T_true^-1."""
    T = np.asarray(T12, np.float64).reshape(3, 4)
    Tt = np.asarray(T_true12, np.float64).reshape(3, 4)
    R = T[:, :3] @ Tt[:, :3].T
    t = T[:, 3] - R @ Tt[:, 3]
    ang = math.acos(max(-1.0, min(1.0, (np.trace(R) - 1.0) / 2.0)))
    return ang, float(np.linalg.norm(t))


def test_c2_pose_gradient_vs_oracle_and_fd(lib, oracle, c2):
    """First tracking step at the perturbed pose: the GPU pose-only gradient (upstream on
    16 crops of 32x32 pixels) against the oracle's analytic gradient, and that gradient
    against FP64 central differences at h = 1e-6 with the fragment decisions frozen."""
    U.log("[gpu] c2 pose gradient vs oracle and finite differences")
    O = oracle
    from paper_2507_03737_amd.render import Rasterizer, Window
    sc = c2
    T0 = scenes.perturb_pose(sc.T_cw[0], 2.0, 0.3, seed=2)
    cam = sc.cams[0]
    params, _ = U.to_dev(sc, torch)
    T = torch.from_numpy(np.ascontiguousarray(T0[None])).cuda()
    cfg = lib.RasterConfig(pointmap_frame=1)
    rast = Rasterizer(Window(sc.cams, T), sc.n, cfg)
    out, fs = rast.forward(params)
    boxes = U.crops(cam, 32, 16, seed=5)
    pix = U.box_pixels(O, boxes)
    view_sc = dataclasses.replace(sc, T_cw=T0[None])
    ref = _check_view_forward(O, view_sc, 0, out, 0, cfg, pixels=pix, tag="c2 crops")
    ok = np.zeros((cam.height, cam.width), bool)
    ok[pix[:, 1], pix[:, 0]] = ref["ambiguous"] == 0
    ups = _upstream(view_sc, 17, [ok], alpha=False)
    up_dev = {k: torch.from_numpy(np.ascontiguousarray(v.reshape(-1))).cuda() for k, v in ups[0].items()}
    pose = torch.zeros(1, 6, device="cuda")
    rast.pose_backward_into(params, out, up_dev, fs, pose)
    torch.cuda.synchronize()
    g_gpu = pose.cpu().numpy()[0].astype(np.float64)

    S = _oracle_settings(O, cfg)
    po = O.Params.from_scene(view_sc)
    view = O.make_view(cam, T0)
    up = O.pixel_upstream(ups[0], pix)
    g_orc = O.backward(po, view, S, pix, up, pointmap_frame=1)["pose"]
    U.log(f"  gpu {g_gpu}\n  oracle {g_orc}")
    U.check_grad("c2 pose", g_gpu, g_orc, frac=1.0)

    tr = O.trace(po, view, S, pix)
    h = 1e-6
    fd = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        lp = O.replay_loss(po, O.make_view(cam, O.se3_exp_left(e, T0)), S, tr, up, 1)
        lm = O.replay_loss(po, O.make_view(cam, O.se3_exp_left(-e, T0)), S, tr, up, 1)
        fd[k] = (lp - lm) / (2 * h)
    U.log(f"  fd {fd}")
    np.testing.assert_allclose(g_orc, fd, rtol=1e-5, atol=1e-5 * np.abs(fd).max())
    assert np.linalg.norm(g_gpu - fd) <= 2e-3 * np.linalg.norm(fd)


def test_c2_tracking_loop_reduces_pose_error(lib, c2):
    """50 pose-only iterations (render -> L1 RGB + L1 pointmap loss -> pose backward ->
    Adam on the se(3) increment -> retract) from a 2 deg / 0.3 m perturbation."""
    U.log("[gpu] c2 tracking loop")
    from paper_2507_03737_amd.render import Rasterizer, Window
    sc = c2
    cam = sc.cams[0]
    params, T_true = U.to_dev(sc, torch)
    cfg = lib.RasterConfig(pointmap_frame=1)
    r_true = Rasterizer(Window(sc.cams, T_true), sc.n, cfg)
    out_t, _ = r_true.forward(params)
    target = out_t["rgb"].clone()
    prior = out_t["pointmap"].clone()
    del r_true
    T0 = scenes.perturb_pose(sc.T_cw[0], 2.0, 0.3, seed=2)
    T = torch.from_numpy(np.ascontiguousarray(T0[None])).cuda()
    win = Window(sc.cams, T)
    rast = Rasterizer(win, sc.n, cfg)
    rast.forward(params)
    rast.max_pairs = int(rast.pairs * 1.5) + 4096
    out = rast.new_outputs()
    fs = rast.new_frame_state()
    scale = torch.empty(win.n_patches(8), device="cuda")
    loss = torch.empty(1, device="cuda")
    g_rgb = torch.empty_like(target)
    g_pm = torch.empty_like(prior)
    pose = torch.zeros(1, 6, device="cuda")
    lr = torch.tensor([0.01, 0.01, 0.01, 0.003, 0.003, 0.003], device="cuda")
    m = torch.zeros(6, device="cuda")
    v = torch.zeros(6, device="cuda")
    b1, b2, eps = 0.9, 0.999, 1e-8
    e0 = _pose_error(T0, sc.T_cw[0])
    losses = []
    for it in range(1, 51):
        rast.forward_into(params, out, fs)
        rast.window_loss_into(out["rgb"], target, out["pointmap"], prior, 8, 0.98, scale, loss, g_rgb, g_pm)
        pose.zero_()
        rast.pose_backward_into(params, out, {"rgb": g_rgb, "pointmap": g_pm}, fs, pose)
        lib.frame_status(fs, lib.stream_handle())
        losses.append(float(loss.item()))
        g = pose[0]
        m.mul_(b1).add_(g, alpha=1 - b1)
        v.mul_(b2).addcmul_(g, g, value=1 - b2)
        step = -lr * (m / (1 - b1 ** it)) / ((v / (1 - b2 ** it)).sqrt() + eps)
        lib.pose_retract(1, T, step[None].contiguous(), lib.stream_handle())
        if it % 10 == 0:
            e = _pose_error(T.cpu().numpy()[0], sc.T_cw[0])
            U.log(f"  it {it}: loss {losses[-1]:.5f} rot {math.degrees(e[0]):.3f} deg trans {e[1]:.4f} m")
    e1 = _pose_error(T.cpu().numpy()[0], sc.T_cw[0])
    U.log(f"  start rot {math.degrees(e0[0]):.3f} deg trans {e0[1]:.4f} m -> "
          f"rot {math.degrees(e1[0]):.3f} deg trans {e1[1]:.4f} m")
    assert losses[-1] < 0.7 * losses[0]
    assert e1[0] < 0.5 * e0[0] and e1[1] < 0.5 * e0[1]
