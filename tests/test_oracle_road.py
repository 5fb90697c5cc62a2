"""Pins of the road-model oracle (fit of Sec. II-C, eq. (11)/(12), and the
disparity transformation of eq. (13)) to facts fixed outside it.

Each pin is chosen so that a plausible slip in the oracle fails one of
them: a sign error in eq. (3) (-u sin(phi)), the centre of the roll
rotation, the branch of phi, a wrong residual in eq. (12), a search that
stops at the wrong minimum, or a transformation with the wrong sign.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import road
from paper_2012_10802_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _plane(a0, a1, phi, W, H):
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    return a0 + a1 * (math.cos(phi) * (v - (H - 1) / 2) - math.sin(phi) * (u - (W - 1) / 2))


def test_hand_worked_3x3():
    """Values worked by hand (tests/golden/hand_road3x3.json)."""
    g = _gold("hand_road3x3.json")
    D = np.array(g["disp"], np.float32)
    f = road.fit_road(D)
    assert f["status"] == 0 and f["count"] == 9
    # phi comes from a 1-D search on a quadratic minimum: good to ~1e-9 rad
    assert f["phi"] == pytest.approx(g["phi"], abs=1e-8)
    for key in ("a0", "a1", "e0min"):
        assert f[key] == pytest.approx(g[key], rel=1e-9, abs=1e-12), key
    u, v, d = road.select(D)
    for p in (0.0, 0.3, g["phi"], -1.2):
        assert road.e0min(u, v, d, p) == pytest.approx(road.residual(u, v, d, p), rel=1e-9, abs=1e-9)
    np.testing.assert_allclose(road.a_of_phi(u, v, d, 0.0), g["a_phi0"], rtol=1e-12)
    assert road.e0min(u, v, d, 0.0) == pytest.approx(g["e0min_phi0"], rel=1e-12)
    D2 = road.transform(D, g["a0"], g["a1"], g["phi"], g["delta_dt"])
    np.testing.assert_allclose(D2, np.array(g["d2"]), rtol=0, atol=1e-6)


@pytest.mark.parametrize("a0,a1,phi_deg", [(30.0, 0.0996, 2.0), (43.6, 0.0996, -3.5),
                                           (12.0, 0.25, 0.0), (80.0, -0.05, 7.0)])
def test_exact_plane_recovered(a0, a1, phi_deg):
    """eq. (3) rendered exactly is fitted back with E0min ~ 0 (rounding of
    the float32 map only); the mask keeps the lower 60 % of the rows, so the
    centring is tested off the selected pixels' mean."""
    W, H = 160, 120
    phi = math.radians(phi_deg)
    D = _plane(a0, a1, phi, W, H).astype(np.float32)
    mask = np.zeros((H, W), np.uint8)
    mask[int(0.4 * H):] = 1
    f = road.fit_road(D, mask)
    assert f["status"] == 0 and f["count"] == mask.sum()
    assert f["phi"] == pytest.approx(phi, abs=1e-6)
    assert f["a1"] == pytest.approx(a1, rel=1e-6)
    assert f["a0"] == pytest.approx(a0, abs=1e-4)
    assert f["e0min"] < 1e-8 * float((D.astype(np.float64) ** 2).sum())


def test_phi_zero_is_the_v_disparity_line():
    """At phi = 0 eq. (11) reduces to eq. (1)/(2), the v-disparity line fit:
    the same as numpy's least-squares polynomial of degree 1 in v."""
    rng = np.random.default_rng(3)
    W, H = 90, 70
    D = (_plane(20.0, 0.1, math.radians(2.5), W, H) + rng.normal(0, 0.4, (H, W))).astype(np.float32)
    u, v, d = road.select(D)
    slope, icpt = np.polyfit(v, d, 1)
    np.testing.assert_allclose(road.a_of_phi(u, v, d, 0.0), [icpt, slope], rtol=1e-10)


def _noisy_scene(W=200, H=150, seed=5, roll=2.0):
    rng = np.random.default_rng(seed)
    D = _plane(25.0, 0.11, math.radians(roll), W, H)
    vv, uu = np.mgrid[0:H, 0:W]
    hole = ((uu - 70) / 25.0) ** 2 + ((vv - 110) / 15.0) ** 2 < 1
    D = np.where(hole, D * 0.94, D) + rng.normal(0, 0.3, (H, W))
    return D.astype(np.float32)


def test_minimum_equals_least_squares_plane():
    """min over phi of eq. (12) is the residual of the least-squares plane
    d ~ c0 + cu u + cv v (numpy lstsq, a different formulation), and eq. (3)
    at the fitted (a, phi) is that plane: -a1 sin(phi) = cu, a1 cos(phi) = cv."""
    D = _noisy_scene()
    f = road.fit_road(D)
    u, v, d = road.select(D)
    A = np.stack([np.ones_like(u), u, v], axis=1)
    coef, res, _, _ = np.linalg.lstsq(A, d, rcond=None)
    assert f["e0min"] == pytest.approx(float(res[0]), rel=1e-9)
    assert -f["a1"] * math.sin(f["phi"]) == pytest.approx(coef[1], rel=1e-7, abs=1e-10)
    assert f["a1"] * math.cos(f["phi"]) == pytest.approx(coef[2], rel=1e-7)
    assert f["a0"] == pytest.approx(coef[0], rel=1e-9)


def test_search_finds_the_global_minimum():
    """E0min at the phi found is below E0min at 200 random angles, and eq.
    (12) has period 180 degrees.  At phi = 0 a rolled road leaves a larger
    residual (the behaviour of Fig. 3); on a full grid u and v are
    uncorrelated, so the excess is exactly the part of d explained by u:
    cov(u, d)^2 / var(u) (sums over the pixels)."""
    D = _noisy_scene(roll=3.0)
    f = road.fit_road(D)
    u, v, d = road.select(D)
    for p in np.random.default_rng(0).uniform(-math.pi, math.pi, 200):
        assert road.e0min(u, v, d, p) >= f["e0min"] * (1 - 1e-12)
    for p in (-1.0, 0.2, 1.3):
        assert road.e0min(u, v, d, p + math.pi) == pytest.approx(road.e0min(u, v, d, p), rel=1e-9)
    uc, dc = u - u.mean(), d - d.mean()
    excess = float(uc @ dc) ** 2 / float(uc @ uc)
    assert road.e0min(u, v, d, 0.0) - f["e0min"] == pytest.approx(excess, rel=1e-7)
    assert excess > 0.3 * f["e0min"]


def test_mirror_flips_the_roll():
    """Mirroring the map left-right (u -> -u about the centre) turns the
    roll into -phi and leaves a0, a1 and E0min unchanged."""
    D = _noisy_scene(roll=2.7)
    f, g = road.fit_road(D), road.fit_road(D[:, ::-1])
    assert g["phi"] == pytest.approx(-f["phi"], abs=1e-8)
    for key in ("a0", "a1", "e0min"):
        assert g[key] == pytest.approx(f[key], rel=1e-8)


def test_selection_and_degenerate_cases():
    D = _noisy_scene()
    # min_disp and NaN drop pixels; an all-zero mask selects nothing
    Dn = D.copy()
    Dn[:10] = np.nan
    assert road.fit_road(Dn)["count"] == D.size - 10 * D.shape[1]
    assert road.fit_road(D, min_disp=1e9)["status"] == 1
    # margin: the match column u - d must stay >= margin
    H, W = D.shape
    for margin in (0.0, 30.5, 100.0):
        want = int((np.arange(W)[None, :] - D.astype(np.float64) >= margin).sum())
        assert road.fit_road(D, margin=margin)["count"] == want
    assert road.fit_road(D, margin=1e9)["status"] == 1
    assert road.fit_road(D, np.zeros(D.shape, np.uint8))["status"] == 1
    two = np.zeros(D.shape, np.uint8)
    two[5, 5] = two[6, 7] = 1
    assert road.fit_road(D, two)["status"] == 1
    # one row, one column, one diagonal: collinear
    for sel in (np.s_[40, :], np.s_[:, 17]):
        m = np.zeros(D.shape, np.uint8)
        m[sel] = 1
        assert road.fit_road(D, m)["status"] == 2
    m = np.zeros(D.shape, np.uint8)
    idx = np.arange(100)
    m[idx, idx] = 1
    f = road.fit_road(D, m)
    assert f["status"] == 2 and math.isnan(f["a0"])


def test_generator_road_is_recovered_and_transformed():
    """On the generator's exact disparity of a rolled road (potholes
    included, road pixels only), the fit recovers the scene's (a0, a1, phi)
    closely, and eq. (13) with the scene's own parameters maps the road to
    delta_DT and the potholes below it (damaged areas stand out)."""
    sc = synth.RoadScene(width=320, height=240, focal=300.0, roll_deg=2.0)
    ps = synth.make_pair(sc, 11)
    a0, a1, phi = ps.road_params
    mask = (ps.road & ~ps.pothole).astype(np.uint8)
    f = road.fit_road(ps.gt.astype(np.float32), mask)
    assert f["status"] == 0
    assert f["phi"] == pytest.approx(phi, abs=1e-6)
    assert f["a1"] == pytest.approx(a1, rel=1e-6)
    assert f["a0"] == pytest.approx(a0, abs=1e-4)
    D2 = road.transform(ps.gt.astype(np.float32), a0, a1, phi, 5.0)
    flat = ps.road & ~ps.pothole
    np.testing.assert_allclose(D2[flat], 5.0, atol=2e-5)
    assert np.all(D2[ps.pothole] < 5.0)


def test_road_mask_is_the_region_below_the_horizon_line():
    """With phi = 0 the road line reaches f_min on the row
    v = cy + (f_min - a0) / a1: the mask is every row below it (closed
    form); a roll tilts that line (a column test), and the margin drops the
    band on the left where the road's match leaves the right image."""
    W, H = 200, 150
    a0, a1 = 10.0, 0.2
    D = _plane(a0, a1, 0.0, W, H).astype(np.float32)
    m = road.road_mask(D, a0, a1, 0.0, 2.0, -np.inf)
    v_h = (H - 1) / 2 + (2.0 - a0) / a1
    rows = np.arange(H) >= v_h
    np.testing.assert_array_equal(m, np.repeat(rows[:, None], W, 1).astype(np.uint8))
    phi = math.radians(5.0)
    m = road.road_mask(D, a0, a1, phi, 2.0, -np.inf)
    assert m[:, 0].sum() > m[:, -1].sum()  # positive roll lifts the road on the left
    m = road.road_mask(D, a0, a1, 0.0, 2.0, 3.0)
    cols = np.arange(W)[None, :]
    f = _plane(a0, a1, 0.0, W, H)
    np.testing.assert_array_equal(m, ((f >= 2.0) & (cols - f >= 3.0)).astype(np.uint8))
    assert m[-1, :28].sum() == 0 and m[-1, 28:].all()  # the bottom row's road disparity is 24.9
    Dn = D.copy()
    Dn[-1, 50] = np.nan
    assert road.road_mask(Dn, a0, a1, 0.0, 2.0, -np.inf)[-1, 50] == 0


def test_refit_on_the_first_fits_road_drops_outliers():
    """A road plane plus an obstacle above the line where the road reaches
    3 px (an eighth of the pixels), at a constant disparity of 5 px that the
    road line never takes there: the plain fit is pulled off the plane; the
    refit over the pixels within 1 px of that first fit equals the fit over
    those pixels chosen directly, and refits converge to the plane.  (With
    a first fit far off the plane, refits can lock onto a wrong band: the
    outliers must be a minority.)"""
    W, H = 240, 160
    a0, a1, phi = 12.0, 0.15, math.radians(2.0)
    plane = _plane(a0, a1, phi, W, H)
    D = np.where(plane >= 3.0, plane, 5.0).astype(np.float32)  # 12.5 % of the pixels
    first = road.fit_road(D, None, 0.5)
    assert abs(first["a1"] - a1) > 0.01
    prior = (first["a0"], first["a1"], first["phi"])
    ref = road.fit_road(D, None, 0.5, prior=prior, tol=1.0)
    near = np.abs(D - road.road_disparity(*prior, W, H)) <= 1.0
    direct = road.fit_road(D, near.astype(np.uint8), 0.5)
    for key in ("a0", "a1", "phi", "e0min", "count"):
        assert ref[key] == pytest.approx(direct[key], rel=1e-12, abs=1e-9)
    for _ in range(3):
        ref = road.fit_road(D, None, 0.5, prior=(ref["a0"], ref["a1"], ref["phi"]), tol=0.25)
    assert ref["phi"] == pytest.approx(phi, abs=1e-6) and ref["a1"] == pytest.approx(a1, rel=1e-6)


def test_window_map_is_the_row_window_at_the_row_centre():
    """The per-pixel windows of the road plane: at the row centre (odd width,
    so cx is a pixel) they equal the C oracle's centred row windows (other
    code, eq. (3) at u = cx); with no roll every column is that row window;
    a roll shifts them by a1 sin(phi) per column."""
    import oracle
    W, H = 161, 120
    for a0, a1, deg in ((14.0, 0.1, 0.0), (20.0, 0.12, 2.5), (30.0, 0.1, -3.0)):
        phi = math.radians(deg)
        lo = road.window_map(a0, a1, phi, W, H, 16)
        rows = oracle.window_from_road(a0, a1, phi, W, H, 16, 0)
        np.testing.assert_array_equal(lo[:, (W - 1) // 2], rows)
        if deg == 0.0:
            np.testing.assert_array_equal(lo, np.repeat(rows[:, None], W, 1))
        else:
            step = np.diff(lo[-1].astype(int))
            assert set(np.unique(step)) <= {0, 1, -1} and abs(step.sum() + a1 * math.sin(phi) * (W - 1)) <= 1
    lo4 = road.window_map(3.0, 0.1, 0.0, 4 * W, 4 * H, 16, scale=4.0)
    np.testing.assert_array_equal(lo4, road.window_map(12.0, 0.1, 0.0, 4 * W, 4 * H, 16))
