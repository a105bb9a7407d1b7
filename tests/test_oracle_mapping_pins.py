"""Pins of the mapping-side oracle (oracle/mapping.py) against closed forms and special
cases: the scale alignment of supplementary Alg. 1, pointmap replacement (Eq. 14), the
isotropic regulariser (Eq. 16), keyframe covisibility (Eq. S1-S2) and the median depth."""
import numpy as np
import pytest

from oracle import mapping as M


def _pointmap(H, W, seed, zlo=5.0, zhi=40.0):
    """Camera-frame points on a smooth random surface (depth zlo..zhi)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    z = zlo + (zhi - zlo) * (0.5 + 0.25 * np.sin(xx / 7.0 + rng.uniform(0, 6)) + 0.2 * np.cos(yy / 5.0))
    z = z + rng.uniform(-0.3, 0.3, (H, W))
    f = 0.8 * W
    return np.stack([(xx - W / 2) * z / f, (yy - H / 2) * z / f, z])


def test_align_exact_global_scale():
    Xp = _pointmap(40, 60, 0)
    Xr = 1.2 * Xp
    r = M.align_scale(Xr, Xp)
    assert r["scale"] == pytest.approx(1.2, rel=1e-12)
    assert r["scales"] == pytest.approx([1.2, 1.2, 1.2], rel=1e-12)
    assert r["cp"] == 40 * 60 and r["n_valid"] == 40 * 60 and not r["insufficient"]


def test_align_excludes_outlier_patches_and_pixels():
    """Inconsistent patches fail the patch test and outlier pixels fail the normalised
    test, so every correct point satisfies |X^r| = s |X^p| and the ratio is exactly s."""
    Xp = _pointmap(50, 70, 1)
    s = 1.15
    Xr = s * Xp
    Xr[:, 10:20, 20:30] *= 3.0            # one whole patch at another scale
    Xr[:, 30:40, 50:60] *= 0.4
    rng = np.random.default_rng(3)
    ys, xs = rng.integers(0, 50, 25), rng.integers(0, 70, 25)
    Xr[:, ys, xs] *= 2.0                   # isolated outlier pixels
    r = M.align_scale(Xr, Xp)
    assert r["scale"] == pytest.approx(s, rel=1e-12)
    assert r["cp"] <= 50 * 70 - 200 - len(set(zip(ys.tolist(), xs.tolist())))


def test_align_without_candidates_keeps_unit_scale():
    Xp = _pointmap(30, 30, 2)
    r = M.align_scale(2.0 * Xp, Xp)        # |mu_r - mu_p| = mu_p > 0.3 mu_p everywhere
    assert r["scale"] == 1.0 and r["cp"] == 0 and r["insufficient"]


def test_align_iterations_admit_patches_as_the_scale_moves():
    """Patches at ratio 1.2 are candidates from the start; patches at 1.45 only once
    sigma' = 1.2 brings them within delta_mu (|1.45 - 1.2| = 0.25 < 0.3 * 1.2).  The
    second estimate is the pooled ratio, and the third iteration keeps it."""
    H, W, P = 40, 40, 10
    Xp = _pointmap(H, W, 4)
    ratio = np.full((H, W), 1.2)
    mid = np.zeros((H, W), bool)
    for py in range(4):
        for px in range(4):
            if (py + px) % 2:
                mid[py * P:(py + 1) * P, px * P:(px + 1) * P] = True
    ratio[mid] = 1.45
    Xr = ratio[None] * Xp
    r = M.align_scale(Xr, Xp, P=P)
    n0 = np.sqrt((Xp * Xp).sum(axis=0))
    pooled = (1.2 * n0[~mid].sum() + 1.45 * n0[mid].sum()) / n0.sum()
    assert r["scales"][0] == pytest.approx(1.2, rel=1e-12)
    assert r["scales"][1] == pytest.approx(pooled, rel=1e-12)
    assert r["scales"][2] == pytest.approx(pooled, rel=1e-12)
    assert r["cp"] == H * W


def test_align_mask_and_partial_border_patches():
    H, W = 33, 47                          # not multiples of P = 10
    Xp = _pointmap(H, W, 5)
    Xr = 0.9 * Xp
    mask = np.ones((H, W))
    mask[::3, ::4] = 0
    Xr[:, ::3, ::4] = 100.0                # garbage where the mask is off
    r = M.align_scale(Xr, Xp, mask=mask)
    assert r["scale"] == pytest.approx(0.9, rel=1e-12)
    assert r["n_valid"] == int(mask.sum()) and r["cp"] == int(mask.sum())


def test_replace_pointmap_closed_form():
    Xp = _pointmap(20, 30, 6)
    s = 1.1
    Xh = s * Xp
    rng = np.random.default_rng(7)
    far = rng.random((20, 30)) < 0.3
    # Offsets of 10% (kept) or 20% (replaced) of |Xh| in a random direction.
    d = rng.standard_normal((3, 20, 30))
    d /= np.sqrt((d * d).sum(axis=0))[None]
    mag = np.where(far, 0.2, 0.1) * np.sqrt((Xh * Xh).sum(axis=0))
    Xr = Xh + d * mag[None]
    out, replaced, margin = M.replace_pointmap(Xr, Xp, s)
    assert np.array_equal(replaced, far)
    np.testing.assert_array_equal(out[:, far], Xh[:, far])
    np.testing.assert_array_equal(out[:, ~far], Xr[:, ~far])
    assert margin > 0.3


def test_iso_loss_closed_form_and_fd():
    ls = np.log(np.array([[1.0], [2.0], [3.0]]))
    loss, g = M.iso_loss(ls)
    assert loss == pytest.approx(2.0, rel=1e-14)
    np.testing.assert_allclose(g[:, 0], [-1.0, 0.0, 3.0], rtol=1e-14, atol=1e-14)
    iso = np.zeros((3, 4))
    loss, g = M.iso_loss(iso)
    assert loss == 0.0 and not g.any()
    rng = np.random.default_rng(8)
    ls = rng.normal(-3.0, 0.7, (3, 50))
    loss, g = M.iso_loss(ls, weight=10.0)
    d = rng.standard_normal(ls.shape)
    h = 1e-6
    fd = (M.iso_loss(ls + h * d, 10.0)[0] - M.iso_loss(ls - h * d, 10.0)[0]) / (2 * h)
    assert fd == pytest.approx((g * d).sum(), rel=1e-6)


def test_covisibility_against_sets():
    rng = np.random.default_rng(9)
    vis = rng.random((5, 200)) < np.array([[0.1], [0.5], [0.5], [0.9], [0.0]])
    iou, oc, counts = M.covisibility(vis)
    sets = [set(np.flatnonzero(v).tolist()) for v in vis]
    for i in range(5):
        assert counts[i] == len(sets[i])
        for j in range(5):
            inter, union = len(sets[i] & sets[j]), len(sets[i] | sets[j])
            assert iou[i, j] == (inter / union if union else 0.0)
            lo = min(len(sets[i]), len(sets[j]))
            assert oc[i, j] == (inter / lo if lo else 0.0)
    assert np.allclose(np.diag(iou)[:4], 1.0) and iou[4, 4] == 0.0
    assert np.array_equal(iou, iou.T) and np.array_equal(oc, oc.T)


def test_median_depth():
    assert M.median_depth(np.array([0.0, 3.0, 1.0, 2.0, 0.0])) == 2.0
    assert M.median_depth(np.array([4.0, 1.0, 3.0, 2.0])) == 2.0      # lower middle
    assert M.median_depth(np.zeros(7)) == 0.0
