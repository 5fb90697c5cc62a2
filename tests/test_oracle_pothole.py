"""Pins of the pothole-threshold oracle (Sec. II-E, eq. (14), (15)) and of
its connected-component labelling, to facts fixed outside it: a
hand-worked map, the unrearranged form of the k-means energy, scipy's
labelling, a two-level map with known potholes and a shift of all values.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import pothole

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_worked_map():
    with open(os.path.join(GOLD, "hand_pothole.json")) as f:
        g = json.load(f)
    D = np.array(g["disp"], np.float32)
    g0, g1, valid = pothole.vectors(D)
    assert valid.sum() == 4 and valid[1, 1:5].all()
    np.testing.assert_array_equal(np.stack([g0[1, 1:5], g1[1, 1:5]], 1), g["g"])
    E2, n1, n2 = pothole.e2_curve(D, g["lo"], g["hi"], g["nbins"])
    eligible = [k for k in range(1, g["nbins"]) if n1[k] > 0 and n2[k] > 0]
    assert eligible == g["eligible"]
    for k, v in g["e2"].items():
        assert E2[int(k)] == v
    t = pothole.threshold(D, g["lo"], g["hi"], g["nbins"], g["delta_pd"])
    assert (t["status"], t["k"], t["t_r"], t["t_s"], t["n1"], t["n2"]) == (0, g["k"], g["t_r"], g["t_s"], g["n1"],
                                                                             g["n2"])
    np.testing.assert_array_equal(pothole.label(D, t["t_s"]), g["labels"])


def test_e2_equals_the_within_cluster_dispersion():
    """eq. (15) is eq. (14) rearranged: sum |g - mu_i|^2 over both regions."""
    rng = np.random.default_rng(1)
    D = (10 + rng.normal(0, 1.0, (40, 50))).astype(np.float32)
    D[10:20, 10:25] -= 4
    lo, hi, nb = 0.0, 16.0, 64
    E2, n1, n2 = pothole.e2_curve(D, lo, hi, nb)
    g0, g1, valid = pothole.vectors(D)
    G = np.stack([g0[valid], g1[valid]], 1)
    i, j = pothole.bins(G[:, 0], G[:, 1], lo, hi, nb)
    checked = 0
    for k in range(1, nb):
        parts = [G[np.maximum(i, j) < k], G[np.minimum(i, j) >= k]]
        if not all(len(p) for p in parts):
            continue
        want = sum(float(((p - p.mean(0)) ** 2).sum()) for p in parts)
        assert E2[k] == pytest.approx(want, rel=1e-9, abs=1e-6)
        checked += 1
    assert checked > 10


def test_labels_match_scipy():
    """8-connected components equal scipy.ndimage.label's, up to naming."""
    from scipy import ndimage
    rng = np.random.default_rng(2)
    for density in (0.2, 0.45, 0.6):
        D = np.where(rng.random((37, 53)) < density, 1.0, 5.0).astype(np.float32)
        lab = pothole.label(D, 3.0)
        ref, n = ndimage.label(D < 3.0, structure=np.ones((3, 3), int))
        assert len(np.unique(lab[lab > 0])) == n
        for c in range(1, n + 1):
            idx = np.flatnonzero(ref.ravel() == c)
            vals = np.unique(lab.ravel()[idx])
            assert vals.tolist() == [idx.min() + 1]
        assert not lab[ref == 0].any()


def _two_level(seed=3, H=120, W=160, road=10.0, depth=6.0):
    rng = np.random.default_rng(seed)
    vv, uu = np.mgrid[0:H, 0:W]
    holes = (((uu - 40) / 18.0) ** 2 + ((vv - 60) / 12.0) ** 2 < 1) | (((uu - 115) / 22.0) ** 2 +
                                                                       ((vv - 80) / 15.0) ** 2 < 1)
    D = np.where(holes, road - depth, road) + rng.normal(0, 0.2, (H, W))
    return D.astype(np.float32), holes


def test_two_level_map_finds_both_potholes():
    D, holes = _two_level()
    t = pothole.threshold(D, 0.0, 16.0, 128, 1.0)
    assert t["status"] == 0 and 4.5 < t["t_r"] < 9.5
    lab = pothole.label(D, t["t_s"])
    names = np.unique(lab[lab > 0])
    assert len(names) == 2
    inter, union = (lab > 0) & holes, (lab > 0) | holes
    assert inter.sum() / union.sum() > 0.9


def test_shift_moves_the_threshold_with_the_values():
    """Adding c (a whole number of bins) to every value and to the range
    shifts t_r by c and leaves the regions, hence n1, n2 and E2, unchanged."""
    D, _ = _two_level(seed=4)
    a = pothole.threshold(D, 0.0, 16.0, 128, 1.0)
    c = 0.125 * 40
    b = pothole.threshold(D + np.float32(c), c, 16.0 + c, 128, 1.0)
    assert (b["k"], b["n1"], b["n2"]) == (a["k"], a["n1"], a["n2"])
    assert b["t_r"] == pytest.approx(a["t_r"] + c, abs=1e-12)
    assert b["e2"] == pytest.approx(a["e2"], rel=1e-6)


def test_masks_borders_and_degenerate_maps():
    D, _ = _two_level(seed=5, H=20, W=30)
    _, _, valid = pothole.vectors(D)
    assert not valid[0].any() and not valid[:, -1].any() and valid[1:-1, 1:-1].all()
    m = np.ones(D.shape, np.uint8)
    m[5, 5] = 0
    _, _, valid = pothole.vectors(D, m)
    assert not valid[4:7, 4:7].any() and valid.sum() == 18 * 28 - 9
    Dn = D.copy()
    Dn[10, 10] = np.nan
    _, _, valid = pothole.vectors(Dn)
    assert not valid[9:12, 9:12].any()
    # a constant map has no split with two non-empty regions
    assert pothole.threshold(np.full((10, 10), 7, np.float32), 0.0, 16.0, 32, 1.0)["status"] == 1
    # maps too small for any vector
    assert pothole.threshold(np.ones((2, 9), np.float32), 0.0, 16.0, 32, 1.0)["status"] == 1
    assert not pothole.label(D, -math.inf).any()


def test_prune_single_superpixel_hand_worked():
    """Sec. III-B: a pothole inside one superpixel counts as false.  Two
    components: the left one lies in superpixel 3 only (removed), the right
    one spans superpixels 4 and 5 (kept with its label)."""
    lab = np.array([[1, 1, 0, 4, 4],
                    [1, 0, 0, 0, 4]], np.int32)
    sp = np.array([[3, 3, 3, 4, 5],
                   [3, 3, 4, 4, 5]], np.int32)
    got = pothole.prune_single_superpixel(lab, sp)
    np.testing.assert_array_equal(got, [[0, 0, 0, 4, 4], [0, 0, 0, 0, 4]])
    # nothing to prune when every component spans two superpixels
    np.testing.assert_array_equal(pothole.prune_single_superpixel(lab, np.arange(10).reshape(2, 5)), lab)
    # everything pruned when the map is one superpixel
    assert not pothole.prune_single_superpixel(lab, np.zeros((2, 5), np.int32)).any()
