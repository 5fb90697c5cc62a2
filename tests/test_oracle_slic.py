"""Pins of the superpixel oracle (SLIC of Sec. II-D, D3 of Sec. II-E) to
facts fixed outside it: hand-worked maps, brute-force nearest centres on a
flat map, D3 against plain per-label means, a two-level map whose potholes
SLIC must keep whole, masks and a value shift.
"""
import json
import os

import numpy as np
import pytest

from oracle import pothole, slic

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_worked_maps():
    with open(os.path.join(GOLD, "hand_slic.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        D = np.array(c["disp"], np.float32)
        Dd, u = slic.used(D)
        ix, iy, iv = slic.init_centres(Dd, u, c["S"])
        np.testing.assert_array_equal(np.stack([ix, iy, iv], 1), c["init"])
        lab, d3, (cx, cy, cv) = slic.slic(D, c["S"], c["m"], c["iters"])
        np.testing.assert_array_equal(lab, c["labels"])
        np.testing.assert_array_equal(np.stack([cx, cy, cv], 1), c["centres"])
        np.testing.assert_array_equal(d3, c["d3"])


def test_flat_map_is_the_nearest_grid_centre():
    """On a constant map centres stay on the grid and one assignment is the
    Voronoi partition of the grid centres (lowest index on a tie), found
    here by brute force over every centre."""
    H, W, S = 37, 50, 8
    D = np.full((H, W), 3.0, np.float32)
    Dd, u = slic.used(D)
    cx, cy, cv = slic.init_centres(Dd, u, S)
    lab = slic.assign(Dd, u, S, 10.0, cx, cy, cv)
    yy, xx = np.mgrid[0:H, 0:W]
    d = (xx[..., None] - cx) ** 2 + (yy[..., None] - cy) ** 2
    np.testing.assert_array_equal(lab, np.argmin(d, axis=-1))


def test_d3_is_the_mean_of_each_superpixel():
    rng = np.random.default_rng(4)
    D = (10 + rng.normal(0, 1.0, (60, 90))).astype(np.float32)
    lab, d3, _ = slic.slic(D, 10, 5.0, 5)
    assert (lab >= 0).all()
    n = lab.max() + 1
    mean = np.bincount(lab.ravel(), D.astype(np.float64).ravel(), n) / np.maximum(np.bincount(lab.ravel(), None, n), 1)
    np.testing.assert_allclose(d3, mean[lab], rtol=0, atol=2.0 ** -20 + 1e-6)
    for k in np.unique(lab):
        assert np.unique(d3[lab == k]).size == 1


def _two_level(seed=3, H=120, W=160):
    rng = np.random.default_rng(seed)
    vv, uu = np.mgrid[0:H, 0:W]
    holes = (((uu - 40) / 18.0) ** 2 + ((vv - 60) / 12.0) ** 2 < 1) | (((uu - 115) / 22.0) ** 2 +
                                                                       ((vv - 80) / 15.0) ** 2 < 1)
    D = np.where(holes, 6.0, 10.0) + rng.normal(0, 0.4, (H, W))
    return D.astype(np.float32), holes


def test_superpixels_follow_pothole_edges_and_detection_improves():
    """SLIC keeps the two depressions apart from the road: few superpixels
    straddle an edge, and thresholding D3 instead of D2 finds the two
    potholes as two components with no noise blobs."""
    D, holes = _two_level()
    lab, d3, _ = slic.slic(D, 8, 2.0, 10)
    mixed = 0
    for k in np.unique(lab):
        frac = holes[lab == k].mean()
        mixed += 0.1 < frac < 0.9
    assert mixed / len(np.unique(lab)) < 0.1
    t = pothole.threshold(D, 0.0, 16.0, 128, 0.5)
    lab3 = pothole.label(d3, t["t_s"])
    assert len(np.unique(lab3[lab3 > 0])) == 2
    found = lab3 > 0
    assert (found & holes).sum() / (found | holes).sum() > 0.85


def test_mask_nan_and_shift():
    D, _ = _two_level(seed=6, H=40, W=48)
    m = np.ones(D.shape, np.uint8)
    m[10:14, 20:30] = 0
    Dn = D.copy()
    Dn[30, 5] = np.nan
    lab, d3, _ = slic.slic(Dn, 6, 3.0, 3, m)
    assert (lab[10:14, 20:30] == -1).all() and lab[30, 5] == -1
    assert np.isnan(d3[10:14, 20:30]).all() and np.isnan(d3[30, 5])
    assert (lab[m.astype(bool) & np.isfinite(Dn)] >= 0).all()
    # a shift of every value by a whole number of quantisation steps keeps the
    # partition and shifts D3 by the same amount
    c = np.float32(4.0)
    lab2, d32, _ = slic.slic(Dn + c, 6, 3.0, 3, m)
    np.testing.assert_array_equal(lab2, lab)
    ok = lab >= 0
    np.testing.assert_allclose(d32[ok], d3[ok] + 4.0, rtol=0, atol=1e-5)


def test_hand_worked_convergence():
    """The stopping rule on the hand-worked maps: the residuals of each
    round and the rounds run at several tolerances, worked by hand; stopping
    at tol = 0 leaves the hand-worked result unchanged."""
    with open(os.path.join(GOLD, "hand_slic.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        D = np.array(c["disp"], np.float32)
        for tol, rounds in c["rounds_at_tol"]:
            info = {}
            lab, d3, (cx, cy, cv) = slic.slic(D, c["S"], c["m"], 10, tol=tol, info=info)
            assert info["rounds"] == rounds, (c["note"][:30], tol)
            np.testing.assert_array_equal(info["residuals"], c["residuals"][:rounds])
            np.testing.assert_array_equal(lab, c["labels"])
            np.testing.assert_array_equal(np.stack([cx, cy, cv], 1), c["centres"])
        info = {}
        slic.slic(D, c["S"], c["m"], 1, tol=0.0, info=info)
        assert info["rounds"] == 1  # never more than `iters`


def test_exact_stop_changes_nothing():
    """Rounds run from the bare steps for a fixed count agree with the
    early-stopped result at tol = 0 whenever the count reaches the stop; a
    positive tol stops no later; residuals are the largest centre moves."""
    D, _ = _two_level(seed=8, H=48, W=64)
    S, m = 8, 2.0
    Dd, u = slic.used(D)
    cx, cy, cv = slic.init_centres(Dd, u, S)
    w = (m / S) ** 2
    moves = []
    for _ in range(40):
        lab = slic.assign(Dd, u, S, m, cx, cy, cv)
        nx, ny, nv, cnt = slic.update(Dd, u, lab, cx, cy, cv)
        e = 0.0
        for k in np.flatnonzero(cnt):
            e = max(e, (nv[k] - cv[k]) ** 2 + ((nx[k] - cx[k]) ** 2 + (ny[k] - cy[k]) ** 2) * w)
        moves.append(e)
        cx, cy, cv = nx, ny, nv
        if e == 0.0:
            break
    assert moves[-1] == 0.0, "this map settles within 40 rounds"
    info = {}
    lab0, d30, (ax, ay, av) = slic.slic(D, S, m, 40, tol=0.0, info=info)
    assert info["rounds"] == len(moves)
    np.testing.assert_array_equal(info["residuals"], moves)
    np.testing.assert_array_equal(np.stack([ax, ay, av]), np.stack([cx, cy, cv]))
    np.testing.assert_array_equal(lab0, lab)
    for tol in (0.05, 0.3, 1.0):
        info = {}
        slic.slic(D, S, m, 40, tol=tol, info=info)
        r = info["rounds"]
        assert all(e > tol * tol for e in moves[:r - 1]) and moves[r - 1] <= tol * tol


def test_centre_without_pixels_does_not_block_the_stop():
    """A centre on a masked-out corner keeps a NaN value and takes no pixels;
    it takes no part in the residual, so the rounds still stop."""
    D = np.array([[1, 1, 5, 5]] * 4, np.float32)
    mask = np.ones((4, 4), np.uint8)
    mask[2:, 2:] = 0
    info = {}
    lab, _, (cx, cy, cv) = slic.slic(D, 2, 0.0, 10, mask, tol=0.0, info=info)
    assert np.isnan(cv).any() and (lab[2:, 2:] == -1).all()
    assert info["rounds"] < 10
