"""GPU (HIP, gfx950) vs FP64 oracle: forward images, tile lists and gradients.

Every test calls the library through its C ABI (via the ctypes binding) on seeded
synthetic inputs and compares with the oracle on the same inputs.
"""
import dataclasses
import math

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


def _posed(sc, deg=3.0, meters=0.1, seed=5):
    sc.T_cw = np.stack([scenes.perturb_pose(T, deg, meters, seed + k) for k, T in enumerate(sc.T_cw)])
    return sc


def _render_gpu(lib, sc, cfg):
    from paper_2507_03737_amd.render import Rasterizer, Window
    params, T = U.to_dev(sc, torch)
    win = Window(sc.cams, T)
    rast = Rasterizer(win, sc.n, cfg)
    out, fs = rast.forward(params)
    torch.cuda.synchronize()
    return rast, params, out, fs


def _oracle_settings(O, cfg):
    return O.Settings(near_z=cfg.near_z, alpha_min=cfg.alpha_min, alpha_max=cfg.alpha_max, t_min=cfg.t_min,
                      eps2d=cfg.eps2d, jac_clamp=cfg.jac_clamp, bg=cfg.bg)


def _check_view_forward(O, sc, v, out, off, cfg, pixels=None, tag="", po=None, proj=None):
    cam = sc.cams[v]
    S = _oracle_settings(O, cfg)
    po = O.Params.from_scene(sc) if po is None else po
    ref, pix = U.oracle_view_images(O, po, cam, sc.T_cw[v], S, pixels, proj=proj)
    ok = ref["ambiguous"] == 0
    key = {0: "pm_world", 1: "pm_cam", 2: "pm_eq5"}[cfg.pointmap_frame]
    host = {k: t.detach().cpu().numpy() for k, t in out.items()}
    got_rgb = U.gpu_pixels(host["rgb"], cam, off, 3, pix)
    got_pm = U.gpu_pixels(host["pointmap"], cam, off, 3, pix)
    U.check_image(f"{tag} rgb", got_rgb.T, ref["rgb"].T, ok[None])
    U.check_image(f"{tag} depth", U.gpu_pixels(host["depth"], cam, off, 1, pix), ref["depth"], ok)
    U.check_image(f"{tag} alpha", U.gpu_pixels(host["alpha"], cam, off, 1, pix), ref["alpha"], ok)
    U.check_image(f"{tag} pointmap", got_pm.T, ref[key].T, ok[None], vector=True)
    return ref


@pytest.mark.parametrize("frame", [0, 1, 2])
def test_forward_c0(lib, oracle, frame):
    U.log(f"[gpu] forward c0 frame={frame}")
    sc = _posed(scenes.make_scene("c0"))
    cfg = lib.RasterConfig(pointmap_frame=frame)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    ref = _check_view_forward(oracle, sc, 0, out, 0, cfg, tag=f"c0/f{frame}")
    assert (ref["ambiguous"] != 0).mean() < 0.01


@pytest.mark.parametrize("tile,ppl", [(8, 1), (16, 1), (16, 2), (16, 4), (32, 1), (32, 2), (32, 4)])
def test_forward_tiles_and_ragged(lib, oracle, tile, ppl):
    """Every launch shape on a view whose size is not a multiple of any tile size."""
    U.log(f"[gpu] forward ragged tile={tile} ppl={ppl}")
    sc = scenes.make_scene("c0", seed=7, n=1500)
    cam = sc.cams[0]
    sc.cams = [scenes.Camera(157, 93, cam.fx, cam.fy, 78.5, 46.5)]
    cfg = lib.RasterConfig(tile=tile, pixels_per_lane=ppl, pointmap_frame=1)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    _check_view_forward(oracle, sc, 0, out, 0, cfg, tag=f"ragged/t{tile}x{ppl}")
    ref = oracle.render_image(oracle.Params.from_scene(sc), sc.cams[0], sc.T_cw[0], _oracle_settings(oracle, cfg))
    up = _upstream(sc, 9, [ref["ambiguous"] == 0])
    g = _gpu_backward(lib, rast, params, out, fs, up)
    r = _oracle_backward(oracle, sc, cfg, up)
    for k in ("means", "log_scales", "quats", "opacity_logit", "rgb"):
        U.check_grad(f"ragged/t{tile}x{ppl} {k}", g[k], r[k])
    U.check_grad(f"ragged/t{tile}x{ppl} pose", g["pose"], r["pose"], frac=1.0)


def test_wave_cull_is_exact(lib):
    """The per-wave rectangle test only skips records that no pixel of the wave accepts:
    at one tile size the per-pixel arithmetic does not depend on the lane layout, so the
    culled layouts (16,1) and (16,2) reproduce the single-wave, unculled (16,4) forward
    bit for bit on a dense street view (c1 size: 300k Gaussians, 1216 x 352)."""
    U.log("[gpu] wave cull exactness c1")
    sc = _posed(scenes.make_scene("c1"))
    sc.cams, sc.T_cw = sc.cams[:1], sc.T_cw[:1]
    outs = {}
    for ppl in (4, 1, 2):
        cfg = lib.RasterConfig(tile=16, pixels_per_lane=ppl, pointmap_frame=1)
        _, _, out, _ = _render_gpu(lib, sc, cfg)
        outs[ppl] = {k: t.detach().cpu().numpy() for k, t in out.items()}
    for ppl in (1, 2):
        for k, ref in outs[4].items():
            assert np.array_equal(outs[ppl][k], ref, equal_nan=True), f"(16,{ppl}) {k}"


def test_sort_digit_widths_agree(lib):
    """The radix sorts are exact and stable at every digit width: 4 to 8 bits per pass (8
    to 4 passes over the 32-bit depth keys, 4 to 2 over the tile ids, so every pass count
    of the histogram, the first-pass scan and the look-back passes runs) give the same
    forward bit for bit on a dense street view (c1 size: 300k Gaussians, 1216 x 352: about
    0.5M tile pairs, so each sort runs over tens of 8192-key tiles); no sort gives up."""
    U.log("[gpu] sort digit widths c1")
    sc = _posed(scenes.make_scene("c1"))
    outs, pairs = {}, {}
    for db in (8, 4, 5, 6, 7):
        cfg = lib.RasterConfig(tile=16, pixels_per_lane=1, pointmap_frame=1, sort_digit_bits=db)
        rast, _, out, fs = _render_gpu(lib, sc, cfg)  # reads the frame status: raises on a stall
        outs[db] = {k: t.detach().cpu().numpy() for k, t in out.items()}
        pairs[db] = rast.pairs
    assert pairs[8] > 20 * 8192, pairs
    for db in (4, 5, 6, 7):
        assert pairs[db] == pairs[8]
        for k, ref in outs[8].items():
            assert np.array_equal(outs[db][k], ref, equal_nan=True), f"digit bits {db}: {k}"


@pytest.mark.parametrize("tile,ppl", [(16, 1), (32, 2)])
def test_contributing_counts_exact(lib, oracle, tile, ppl):
    """Per-pixel counts of contributing fragments (alpha >= alpha_min before the
    transmittance floor) equal the oracle's, bit for bit, wherever no decision lies within
    rounding of its threshold; the work query reports their sum and refuses a frame state
    whose forward did not count.  Its accepted (wave, entry) count equals the bits of the
    per-wave planes, and bounds the walked count from below and F / 64 from above."""
    U.log(f"[gpu] contributing counts c0 tile {tile} ppl {ppl}")
    sc = _posed(scenes.make_scene("c0"))
    cam = sc.cams[0]
    cfg = lib.RasterConfig(pointmap_frame=1, tile=tile, pixels_per_lane=ppl)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    with pytest.raises(lib.GspmError):
        rast.work(fs)
    cfg.count_work = 1
    out, fs = rast.forward(params)
    torch.cuda.synchronize()
    pairs, frags, _, walked, accepted = rast.work(fs)
    n_tiles = math.ceil(cam.width / tile) * math.ceil(cam.height / tile)
    lay = U.frame_layout(n_tiles, cam.width * cam.height, sc.n)
    raw = fs.cpu().numpy()
    got = raw[lay["contrib"]:lay["contrib"] + 4 * cam.width * cam.height].view(np.uint32)
    got = got.reshape(cam.height, cam.width)
    S = _oracle_settings(oracle, cfg)
    ref, _ = U.oracle_view_images(oracle, oracle.Params.from_scene(sc), cam, sc.T_cw[0], S, None)
    ok = (ref["ambiguous"] == 0).reshape(cam.height, cam.width)
    n_ref = ref["n_frag"].reshape(cam.height, cam.width)
    bad = int((got[ok] != n_ref[ok]).sum())
    U.log(f"  fragments {frags} (oracle {int(n_ref.sum())}), pixels checked {int(ok.sum())}, mismatches {bad}")
    assert bad == 0
    assert frags == int(got.astype(np.int64).sum())
    # The accepted (wave, entry) count is the number of bits in the per-wave planes; every
    # contributing fragment lies in an accepted entry of its pixel's wave.
    cap = int(raw[lay["header"]:lay["header"] + 16].view(np.uint32)[2])
    a = lambda x: (x + 255) & ~255  # noqa: E731
    w0 = lay["pair_vals"] + a(4 * cap)
    planes = tile * tile // ppl // 64  # one plane per wave of the forward (the rest is not cleared)
    words = raw[w0:w0 + 8 * planes * (cap // 64 + 2)].view(np.uint64)
    bits = int(np.unpackbits(words.view(np.uint8)).sum())
    U.log(f"  walked {walked}, accepted {accepted} (bits {bits}), 64 x accepted / F = {64 * accepted / frags:.2f}")
    assert accepted == bits
    assert walked >= accepted and 64 * accepted >= frags


def test_launch_orders(lib):
    """The forward and backward launch orders are permutations of the tiles, heaviest
    first: non-increasing in list length (forward) and in the deepest contributing list
    entry of the tile (backward), in classes of 32 entries."""
    U.log("[gpu] launch orders c1")
    sc = _posed(scenes.make_scene("c1"))
    cfg = lib.RasterConfig(pointmap_frame=1, tile=16, pixels_per_lane=1)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    cam = sc.cams[0]
    n_tiles = math.ceil(cam.width / 16) * math.ceil(cam.height / 16) * len(sc.cams)
    npix = sum(c.width * c.height for c in sc.cams)
    assert all((c.width, c.height) == (cam.width, cam.height) for c in sc.cams)
    lay = U.frame_layout(n_tiles, npix, sc.n * len(sc.cams))
    raw = fs.cpu().numpy()
    ranges = raw[lay["ranges"]:lay["ranges"] + 8 * n_tiles].view(np.uint32).reshape(n_tiles, 2)
    order = raw[lay["order"]:lay["order"] + 8 * n_tiles].view(np.uint32).reshape(2, n_tiles)
    last = raw[lay["last"]:lay["last"] + 4 * npix].view(np.uint32)
    for o in order:
        assert np.array_equal(np.sort(o), np.arange(n_tiles, dtype=np.uint32))
    cls = lambda w: np.minimum(w.astype(np.int64) >> 5, 255)  # noqa: E731
    assert np.all(np.diff(cls(ranges[order[0], 1] - ranges[order[0], 0])) <= 0)
    # Deepest contributing entry per tile, from the per-pixel counts.
    tx, ty = math.ceil(cam.width / 16), math.ceil(cam.height / 16)
    deep = []
    for v in range(len(sc.cams)):
        img = last[v * cam.width * cam.height:(v + 1) * cam.width * cam.height].reshape(cam.height, cam.width)
        pad = np.zeros((ty * 16, tx * 16), np.uint32)
        pad[:cam.height, :cam.width] = img
        deep.append(pad.reshape(ty, 16, tx, 16).max(axis=(1, 3)).reshape(-1))
    deep = np.concatenate(deep)
    assert np.all(np.diff(cls(deep[order[1]])) <= 0)


@pytest.mark.parametrize("tile,ppl", [(16, 2), (8, 1), (32, 1)])
def test_tile_lists_between_exact_and_rect(lib, oracle, tile, ppl):
    """Per-tile record lists against the oracle's two definitions of a tile's Gaussians
    (the tile-based rasterization of Sec. 3.1): every Gaussian with a pixel centre of the
    tile where its alpha reaches alpha_min (exact) is listed, and every listed Gaussian has
    a pixel of its support box in the tile (rect); lists are ordered by (float32 depth,
    index).  Exempt are decisions taken at an edge: an exact pair whose nearest pixel
    centre lies within 1e-5 (relative) of the support level, and a listed pair outside the
    rect whose box bound lies within 1e-4 px (plus the float32 rounding of the record) of
    a tile edge.  The surplus over the exact lists is reported."""
    U.log(f"[gpu] tile lists c0 tile {tile} ppl {ppl}")
    O = oracle
    sc = _posed(scenes.make_scene("c0"))
    cfg = lib.RasterConfig(pointmap_frame=1, tile=tile, pixels_per_lane=ppl)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    cam = sc.cams[0]
    B = cfg.tile
    n_tiles = math.ceil(cam.width / B) * math.ceil(cam.height / B)
    lay = U.frame_layout(n_tiles, cam.width * cam.height, sc.n)
    raw = fs.cpu().numpy()
    pairs = int(raw[:4].view(np.uint32)[0])
    ranges = raw[lay["ranges"]:lay["ranges"] + 8 * n_tiles].view(np.uint32).reshape(n_tiles, 2)
    vals = raw[lay["pair_vals"]:lay["pair_vals"] + 4 * pairs].view(np.uint32)
    S = _oracle_settings(O, cfg)
    po = O.Params.from_scene(sc)
    proj = O.project(po, O.make_view(cam, sc.T_cw[0]), S)
    pa = O.proj_numpy(proj)
    tiles_o, gs_o, ratio = O.tile_sets(proj, po.n, cam.width, cam.height, B, S)
    tol_px = 1e-4 + 2e-7 * (np.abs(pa["u"]) + np.abs(pa["v"]) + pa["rx"] + pa["ry"])
    edge = U.tile_edge_near(pa["bounds"], B, cam.width, cam.height, tol_px) & (pa["visible"] == 1)
    z32 = pa["z"].astype(np.float32)
    exact = ratio <= 1.0
    near = np.abs(ratio - 1.0) <= 1e-5
    n_exact = n_surplus = n_near_missing = 0
    for t in range(n_tiles):
        got = [int(x) for x in vals[ranges[t, 0]:ranges[t, 1]]]
        assert got == sorted(got, key=lambda g: (z32[g], g)), f"tile {t}: not in (float32 depth, index) order"
        got_set = set(got)
        sel = tiles_o == t
        must = set(gs_o[sel & exact & ~near].tolist())
        may = set(gs_o[sel].tolist())
        missing = must - got_set
        assert not missing, f"tile {t}: exact pairs not listed {sorted(missing)[:8]}"
        outside = {g for g in got_set - may if not edge[g]}
        assert not outside, f"tile {t}: listed Gaussians outside their support box {sorted(outside)[:8]}"
        n_exact += int((sel & exact).sum())
        n_surplus += len(got_set - set(gs_o[sel & exact].tolist()))
        n_near_missing += len(set(gs_o[sel & exact & near].tolist()) - got_set)
    U.log(f"  pairs={pairs} exact={n_exact} rect={len(tiles_o)} surplus over exact={n_surplus} "
          f"({n_surplus / max(1, n_exact):.1%}) exempt near-level pairs missing={n_near_missing}")


def _upstream(sc, seed, ok_masks, alpha=True):
    ups = scenes.upstream_grads(sc, seed=seed, alpha=alpha)
    for up, ok in zip(ups, ok_masks):
        for k in ("rgb", "pointmap"):
            up[k] = np.ascontiguousarray(up[k] * ok[None])
        for k in ("depth", "alpha"):
            up[k] = np.ascontiguousarray(up[k] * ok)
    return ups


def _pack(ups, key, channels):
    return np.concatenate([u[key].reshape(-1) for u in ups]).astype(np.float32)


def _gpu_backward(lib, rast, params, out, fs, ups, pose=True):
    up = {k: torch.from_numpy(_pack(ups, k, c)).cuda() for k, c in (("rgb", 3), ("depth", 1), ("alpha", 1),
                                                                     ("pointmap", 3))}
    grads = rast.zero_grads(params)
    pg = torch.zeros(rast.win.n_views, 6, device="cuda") if pose else None
    rast.backward_into(params, out, up, fs, grads, pg)
    torch.cuda.synchronize()
    g = {k: t.cpu().numpy() for k, t in grads.items()}
    if pose:
        g["pose"] = pg.cpu().numpy()
    return g


def _oracle_backward(O, sc, cfg, ups, pixel_sets=None, po=None, projs=None):
    S = _oracle_settings(O, cfg)
    po = O.Params.from_scene(sc) if po is None else po
    tot = None
    poses = []
    for v, cam in enumerate(sc.cams):
        pix = O.full_pixels(cam) if pixel_sets is None else pixel_sets[v]
        view = O.make_view(cam, sc.T_cw[v])
        up = O.pixel_upstream(ups[v], pix)
        g = O.backward(po, view, S, pix, up, pointmap_frame=cfg.pointmap_frame,
                       proj=None if projs is None else projs[v])
        poses.append(g.pop("pose"))
        tot = g if tot is None else {k: tot[k] + g[k] for k in tot}
    tot["pose"] = np.stack(poses)
    return tot


@pytest.mark.parametrize("lane_reduce", [0, 1])
@pytest.mark.parametrize("frame", [0, 1, 2])
def test_backward_c0(lib, oracle, frame, lane_reduce):
    """Gradients against the oracle, with the per-record sums on the matrix cores
    (lane_reduce=0) and with the cross-lane reduce-scatter (lane_reduce=1)."""
    U.log(f"[gpu] backward c0 frame={frame} lane_reduce={lane_reduce}")
    O = oracle
    sc = _posed(scenes.make_scene("c0"))
    cfg = lib.RasterConfig(pointmap_frame=frame, bwd_lane_reduce=lane_reduce)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    ref = O.render_image(O.Params.from_scene(sc), sc.cams[0], sc.T_cw[0], _oracle_settings(O, cfg))
    ups = _upstream(sc, 21, [ref["ambiguous"] == 0])
    g = _gpu_backward(lib, rast, params, out, fs, ups)
    r = _oracle_backward(O, sc, cfg, ups)
    for k in ("means", "log_scales", "quats", "opacity_logit", "rgb"):
        rel = U.check_grad(f"c0/f{frame} {k}", g[k], r[k])
        U.log(f"  {k}: rel {rel:.2e}")
    U.check_grad(f"c0/f{frame} pose", g["pose"], r["pose"], frac=1.0)
    U.log(f"  pose gpu {g['pose'][0]} oracle {r['pose'][0]}")


@pytest.mark.parametrize("pose_only", [False, True])
def test_grads_overwrite(lib, pose_only):
    """With settings.grads_overwrite the backward writes the parameter and pose gradients
    over whatever the arrays held (NaN here): what it adds into zeroed arrays, up to the
    order of the float atomics that sum each record's image-plane terms (which differs
    from run to run), and zeros for Gaussians that get none."""
    U.log(f"[gpu] gradients written over the arrays, pose_only={pose_only}")
    sc = _posed(scenes.make_scene("c0"))
    sc.opacity_logit[:50] = -30.0  # Gaussians below alpha_min everywhere: no gradient flows to them
    cfg = lib.RasterConfig(pointmap_frame=1)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    ups = _upstream(sc, 23, [np.ones((sc.cams[0].height, sc.cams[0].width), dtype=bool)])
    up = {k: torch.from_numpy(_pack(ups, k, c)).cuda() for k, c in (("rgb", 3), ("depth", 1), ("alpha", 1),
                                                                     ("pointmap", 3))}
    res = []
    for overwrite in (False, True):
        fill = float("nan") if overwrite else 0.0
        grads = {k: torch.full_like(t, fill) for k, t in rast.zero_grads(params).items()}
        pg = torch.full((1, 6), fill, device="cuda")
        if pose_only:
            c = dataclasses.replace(rast.cfg, grads_overwrite=int(overwrite))
            saved, rast.cfg = rast.cfg, c
            rast.pose_backward_into(params, out, up, fs, pg)
            rast.cfg = saved
        else:
            rast.backward_into(params, out, up, fs, grads, pg, overwrite=overwrite)
        torch.cuda.synchronize()
        res.append(({k: t.cpu().numpy() for k, t in grads.items()}, pg.cpu().numpy()))
    (g0, p0), (g1, p1) = res

    def same(a, b, tag):
        assert np.isfinite(b).all(), tag
        assert np.allclose(a, b, rtol=1e-5, atol=1e-6 * float(np.abs(a).max())), tag

    same(p0, p1, "pose")
    if not pose_only:
        for k in g0:
            same(g0[k], g1[k], k)
        assert not np.any(g1["means"][:, :50]) and not np.any(g1["opacity_logit"][:50])


@pytest.mark.parametrize("tile,ppl", [(8, 1), (16, 1), (16, 2), (16, 4), (32, 1), (32, 2), (32, 4)])
def test_backward_shapes(lib, oracle, tile, ppl):
    """Gradients against the oracle for every launch shape of the raster kernels: the
    matrix-core backward (one pixel per lane: 1, 4 or 16 waves per tile) and the
    reduce-scatter backward (2 and 4 pixels per lane)."""
    U.log(f"[gpu] backward c0 tile={tile} ppl={ppl}")
    O = oracle
    sc = _posed(scenes.make_scene("c0"))
    cfg = lib.RasterConfig(pointmap_frame=1, tile=tile, pixels_per_lane=ppl)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    ref = O.render_image(O.Params.from_scene(sc), sc.cams[0], sc.T_cw[0], _oracle_settings(O, cfg))
    ups = _upstream(sc, 24, [ref["ambiguous"] == 0])
    g = _gpu_backward(lib, rast, params, out, fs, ups)
    r = _oracle_backward(O, sc, cfg, ups)
    for k in ("means", "log_scales", "quats", "opacity_logit", "rgb"):
        U.check_grad(f"c0 {tile}x{tile}/ppl{ppl} {k}", g[k], r[k])
    U.check_grad(f"c0 {tile}x{tile}/ppl{ppl} pose", g["pose"], r["pose"], frac=1.0)


def test_zero_quaternions(lib, oracle):
    """Gaussians whose quaternion cannot be normalised are dropped from every view (the
    view-independent part of the projection fails once per Gaussian): forward and backward
    still match the oracle, and those Gaussians get no gradient."""
    U.log("[gpu] c0 with zero quaternions")
    O = oracle
    sc = _posed(scenes.make_scene("c0"))
    dead = np.arange(0, sc.quats.shape[1], 7)
    sc.quats[:, dead] = 0.0
    cfg = lib.RasterConfig(pointmap_frame=1)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    _check_view_forward(O, sc, 0, out, 0, cfg, tag="c0/zero-quats")
    ref = O.render_image(O.Params.from_scene(sc), sc.cams[0], sc.T_cw[0], _oracle_settings(O, cfg))
    ups = _upstream(sc, 31, [ref["ambiguous"] == 0])
    g = _gpu_backward(lib, rast, params, out, fs, ups)
    r = _oracle_backward(O, sc, cfg, ups)
    for k in ("means", "log_scales", "quats", "opacity_logit", "rgb"):
        assert np.all(g[k][..., dead] == 0.0), k
        U.check_grad(f"c0 zero-quats {k}", g[k], r[k])
    U.check_grad("c0 zero-quats pose", g["pose"], r["pose"], frac=1.0)


@pytest.mark.parametrize("ppl_fwd,ppl_bwd", [(2, 1), (1, 2)])
def test_backward_after_forward_with_other_shape(lib, oracle, ppl_fwd, ppl_bwd):
    """A backward whose pixels per lane differ from its forward's: the forward's per-wave
    contribution bits follow other waves, so the backward culls instead; gradients still
    match the oracle."""
    U.log(f"[gpu] backward c0 forward ppl={ppl_fwd} backward ppl={ppl_bwd}")
    O = oracle
    sc = _posed(scenes.make_scene("c0"))
    cfg = lib.RasterConfig(pointmap_frame=1, pixels_per_lane=ppl_fwd)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    ref = O.render_image(O.Params.from_scene(sc), sc.cams[0], sc.T_cw[0], _oracle_settings(O, cfg))
    ups = _upstream(sc, 23, [ref["ambiguous"] == 0])
    rast.cfg.pixels_per_lane = ppl_bwd
    g = _gpu_backward(lib, rast, params, out, fs, ups)
    r = _oracle_backward(O, sc, cfg, ups)
    for k in ("means", "log_scales", "quats", "opacity_logit", "rgb"):
        U.check_grad(f"c0 ppl {ppl_fwd}->{ppl_bwd} {k}", g[k], r[k])
    U.check_grad(f"c0 ppl {ppl_fwd}->{ppl_bwd} pose", g["pose"], r["pose"], frac=1.0)


@pytest.mark.parametrize("lane_reduce", [0, 1])
def test_pose_backward_matches_full_backward(lib, oracle, lane_reduce):
    U.log(f"[gpu] pose-only backward c0 lane_reduce={lane_reduce}")
    sc = _posed(scenes.make_scene("c0"))
    cfg = lib.RasterConfig(pointmap_frame=1, bwd_lane_reduce=lane_reduce)
    rast, params, out, fs = _render_gpu(lib, sc, cfg)
    ref = oracle.render_image(oracle.Params.from_scene(sc), sc.cams[0], sc.T_cw[0], _oracle_settings(oracle, cfg))
    ups = _upstream(sc, 22, [ref["ambiguous"] == 0])
    up = {k: torch.from_numpy(_pack(ups, k, c)).cuda() for k, c in (("rgb", 3), ("depth", 1), ("alpha", 1),
                                                                     ("pointmap", 3))}
    pg = torch.zeros(1, 6, device="cuda")
    rast.pose_backward_into(params, out, up, fs, pg)
    torch.cuda.synchronize()
    r = _oracle_backward(oracle, sc, cfg, ups)
    U.check_grad("pose-only", pg.cpu().numpy(), r["pose"], frac=1.0)


def test_empty_and_culled(lib, oracle):
    """No Gaussians, and Gaussians that are all behind the camera: background only."""
    U.log("[gpu] empty / all culled")
    from paper_2507_03737_amd.render import Rasterizer, Window
    cam = scenes.Camera(40, 30, 30.0, 30.0, 20.0, 15.0)
    T = torch.tensor(np.eye(3, 4, dtype=np.float32).reshape(1, 12)).cuda()
    cfg = lib.RasterConfig(bg=(0.25, 0.5, 0.75))
    win = Window([cam], T)
    for n in (0, 50):
        sc = scenes.make_scene("c0", seed=3, n=max(n, 1))
        params = [torch.from_numpy(np.ascontiguousarray(a[..., :n])).cuda() for a in sc.params()]
        if n:
            params[0][2] = -5.0  # behind the camera
        rast = Rasterizer(win, n, cfg)
        out, fs = rast.forward(params)
        assert rast.pairs == 0
        rgb = out["rgb"].view(3, 30, 40).cpu().numpy()
        for c, b in enumerate(cfg.bg):
            assert np.all(rgb[c] == np.float32(b))
        assert float(out["alpha"].abs().max()) == 0.0 and float(out["depth"].abs().max()) == 0.0
        up = {"rgb": torch.ones(3 * 1200, device="cuda")}
        grads = rast.zero_grads(params)
        pg = torch.zeros(1, 6, device="cuda")
        rast.backward_into(params, out, up, fs, grads, pg)
        torch.cuda.synchronize()
        assert all(float(t.abs().max()) == 0.0 for t in grads.values() if t.numel()) and float(pg.abs().max()) == 0.0


def test_capacity_overflow_reports_and_recovers(lib):
    U.log("[gpu] capacity overflow")
    from paper_2507_03737_amd.render import Rasterizer, Window
    sc = scenes.make_scene("c0")
    params, T = U.to_dev(sc, torch)
    rast = Rasterizer(Window(sc.cams, T), sc.n, lib.RasterConfig(), max_pairs=100)
    out = rast.new_outputs()
    fs = rast.new_frame_state()
    rast.forward_into(params, out, fs)
    with pytest.raises(lib.CapacityError) as ei:
        lib.frame_status(fs, lib.stream_handle())
    need = ei.value.pairs
    assert need > 100
    out2, fs2 = rast.forward(params)  # grows and retries
    assert rast.pairs == need and rast.max_pairs >= need


def test_backward_refuses_a_mismatched_or_incomplete_frame(lib):
    """A backward whose tile or pointmap frame differs from its forward's, or that follows
    a forward whose pair list overflowed, reads nothing of the frame state: it adds no
    gradient and gspm_frame_status reports the refusal until the next forward."""
    U.log("[gpu] backward refuses a mismatched frame state")
    import dataclasses
    from paper_2507_03737_amd.render import Rasterizer, Window
    sc = _posed(scenes.make_scene("c0", n=500))
    params, T = U.to_dev(sc, torch)
    up = {"rgb": torch.ones(3 * 160 * 120, device="cuda"), "pointmap": torch.ones(3 * 160 * 120, device="cuda")}
    for field, value in (("tile", 8), ("pointmap_frame", 0)):
        rast = Rasterizer(Window(sc.cams, T), sc.n, lib.RasterConfig(tile=16, pointmap_frame=1))
        out, fs = rast.forward(params)
        rast.cfg = dataclasses.replace(rast.cfg, **{field: value})
        grads = rast.zero_grads(params)
        pg = torch.zeros(1, 6, device="cuda")
        rast.backward_into(params, out, up, fs, grads, pg)
        torch.cuda.synchronize()
        assert all(float(t.abs().max()) == 0.0 for t in grads.values()) and float(pg.abs().max()) == 0.0, field
        with pytest.raises(lib.GspmError) as ei:
            lib.frame_status(fs, lib.stream_handle())
        assert ei.value.status == lib.GSPM_ERR_INVALID_ARG and "refused" in str(ei.value), field
        rast.cfg = dataclasses.replace(rast.cfg, **{field: {"tile": 16, "pointmap_frame": 1}[field]})
        out, fs = rast.forward(params)  # a new forward clears the mark; the matching backward runs
        rast.backward_into(params, out, up, fs, grads, pg)
        assert lib.frame_status(fs, lib.stream_handle()) > 0
        assert float(grads["means"].abs().max()) > 0.0
    rast = Rasterizer(Window(sc.cams, T), sc.n, lib.RasterConfig(), max_pairs=100)
    out, fs = rast.new_outputs(), rast.new_frame_state()
    rast.forward_into(params, out, fs)
    grads = rast.zero_grads(params)
    rast.backward_into(params, out, up, fs, grads, None)
    torch.cuda.synchronize()
    assert all(float(t.abs().max()) == 0.0 for t in grads.values())
    with pytest.raises(lib.CapacityError):
        lib.frame_status(fs, lib.stream_handle())
