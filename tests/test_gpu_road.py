"""Parity of the road-model calls (fit of Sec. II-C, windows of eq. (6),
transformation of eq. (13)) with the CPU oracle, through the C ABI.

Tolerances (float64 on both sides; the oracle searches phi, the library
solves in closed form):
  count           exact (sums of integers stay exact in float64);
  phi             1e-7 rad   (the oracle's golden-section search resolves
                              a quadratic minimum to ~1e-9 rad);
  a1              1e-7 relative, a0 1e-5 px (follow from phi);
  e0min           1e-6 relative, or 1e-10 of sum d^2 when the residual is
                  ~0 (the one-pass moments subtract sums of size sum d^2);
  window starts   equal, except where the oracle's value before floor()
                  lies within 1e-6 of an integer;
  transformation  one float32 rounding of float64 values that agree to
                  ~1e-14: 2.5e-7 relative (one ulp).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import road as oroad
from paper_2012_10802_amd import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def lib():
    import torch
    from paper_2012_10802_amd import sgm
    assert torch.cuda.is_available()
    return sgm


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _close_fit(got, want, D):
    assert got["status"] == want["status"]
    assert got["count"] == want["count"]
    if want["status"] != 0:
        for k in ("a0", "a1", "phi", "e0min"):
            assert math.isnan(got[k])
        return
    assert got["phi"] == pytest.approx(want["phi"], abs=1e-7)
    assert got["a1"] == pytest.approx(want["a1"], rel=1e-7)
    assert got["a0"] == pytest.approx(want["a0"], abs=1e-5)
    sdd = float(np.nansum(np.where(np.isfinite(D), D.astype(np.float64), 0.0) ** 2))
    assert got["e0min"] == pytest.approx(want["e0min"], rel=1e-6, abs=1e-10 * sdd)
    assert got["g_u"] == pytest.approx(-got["a1"] * math.sin(got["phi"]), rel=1e-9, abs=1e-15)
    assert got["g_v"] == pytest.approx(got["a1"] * math.cos(got["phi"]), rel=1e-9, abs=1e-15)


def _fit_one(lib, D, mask=None, min_disp=-math.inf, margin=-math.inf):
    fit = lib.road_fit(_dev(D), None if mask is None else _dev(mask.astype(np.uint8)), min_disp, margin)
    return lib.road_fit_dicts(fit)[0], fit


def test_hand_worked_3x3(lib):
    """The hand-worked map (odd width: the one-pixel-per-load path)."""
    with open(os.path.join(GOLD, "hand_road3x3.json")) as f:
        g = json.load(f)
    D = np.array(g["disp"], np.float32)
    got, fit = _fit_one(lib, D)
    assert got["status"] == 0 and got["count"] == 9
    for k in ("a0", "a1", "phi", "e0min"):
        assert got[k] == pytest.approx(g[k], rel=1e-12, abs=1e-12), k
    D2 = lib.disparity_transform(_dev(D), fit, g["delta_dt"]).cpu().numpy()
    np.testing.assert_allclose(D2, np.array(g["d2"]), rtol=0, atol=1e-6)


def _sgm_disp(lib, cfg, seed):
    import torch
    sc = synth.scene_for_config(cfg, seed)
    ps = synth.make_pair(sc, seed)
    c = synth.CONFIGS[cfg]
    m = lib.Matcher(sc.width, sc.height, census=c["census"], ndisp=c["ndisp"], npaths=c["npaths"],
                    p1=c["p1"], p2=c["p2"])
    _, ds = m.match(_dev(ps.left), _dev(ps.right))
    torch.cuda.synchronize()
    return ps, ds.cpu().numpy()


@pytest.mark.parametrize("cfg,seed", [("road320", 2), ("road640", 7)])
def test_fit_on_sgm_output_matches_oracle(lib, cfg, seed):
    """Fit to the library's own SGM disparity of a generated road pair, road
    pixels only (the generator's road mask), both with and without a mask,
    with a disparity floor."""
    ps, D = _sgm_disp(lib, cfg, seed)
    mask = ps.road
    got, _ = _fit_one(lib, D, mask)
    _close_fit(got, oroad.fit_road(D, mask), D)
    got, _ = _fit_one(lib, D, None, 0.5)
    _close_fit(got, oroad.fit_road(D, None, 0.5), D)
    # matches inside the right image only (the selection a pipeline without
    # ground truth can make)
    for margin in (4.0, 10.5):
        got, _ = _fit_one(lib, D, None, 0.5, margin)
        _close_fit(got, oroad.fit_road(D, None, 0.5, margin), D)
    # on the scored road pixels (matchable, away from the borders, no
    # potholes) the fit lands near the scene's own road line
    a0, a1, phi = ps.road_params
    r = synth.CONFIGS[cfg]["census"] // 2
    H, W = D.shape
    good = ps.road & ~ps.pothole & (np.arange(W)[None, :] - ps.gt >= r + 2)
    good[:r] = good[-r:] = False
    good[:, :r] = good[:, -r:] = False
    got, _ = _fit_one(lib, D, good)
    _close_fit(got, oroad.fit_road(D, good), D)
    assert abs(got["phi"] - phi) < 2e-3 and abs(got["a1"] - a1) < 2e-3


@pytest.mark.parametrize("W,H", [(257, 131), (64, 1000), (1, 50), (50, 1), (4, 3), (1283, 37),
                                 (1024, 7), (1028, 6), (2600, 9), (4100, 5)])
def test_fit_shapes_and_batches(lib, W, H):
    """Ragged widths (one pixel per access), widths divisible by 4 up to 1024,
    2048 and 4096 (float4 paths with 1, 2, 4 groups per thread and row) and
    beyond, odd and even row counts, single rows / columns (degenerate),
    several maps per launch with NaN, infinite and below-floor pixels and
    masks; the transformation on the same maps."""
    rng = np.random.default_rng(W * 1000 + H)
    n = 3
    Ds, Ms = [], []
    for i in range(n):
        D = oroad.road_disparity(20 + 5 * i, 0.1 + 0.02 * i, math.radians(1.5 - i), W, H)
        D = (D + rng.normal(0, 0.5, (H, W))).astype(np.float32)
        D.flat[rng.integers(0, D.size, max(1, D.size // 50))] = np.nan
        D.flat[rng.integers(0, D.size, max(1, D.size // 100))] = np.inf
        Ds.append(D)
        Ms.append((rng.random((H, W)) < 0.8).astype(np.uint8))
    Ds, Ms = np.stack(Ds), np.stack(Ms)
    fits = lib.road_fit_dicts(lib.road_fit(_dev(Ds), _dev(Ms), 19.0))
    for i in range(n):
        _close_fit(fits[i], oroad.fit_road(Ds[i], Ms[i], 19.0), Ds[i])
    margin = W / 3 - 20.25
    fits = lib.road_fit_dicts(lib.road_fit(_dev(Ds), _dev(Ms), -math.inf, margin))
    for i in range(n):
        _close_fit(fits[i], oroad.fit_road(Ds[i], Ms[i], -math.inf, margin), Ds[i])
    fit = lib.road_fit(_dev(Ds))
    fits = lib.road_fit_dicts(fit)
    for i in range(n):
        _close_fit(fits[i], oroad.fit_road(Ds[i]), Ds[i])
    D2 = lib.disparity_transform(_dev(Ds), fit, 4.0).cpu().numpy()
    for i in range(n):
        f = fits[i]
        if f["status"] == 0:
            want = oroad.transform(Ds[i], f["a0"], f["a1"], f["phi"], 4.0)
            np.testing.assert_allclose(D2[i], want, rtol=2.5e-7, atol=1e-9)
        else:
            assert np.isnan(D2[i]).all()


def test_degenerate_selections(lib):
    H, W = 40, 64
    D = oroad.road_disparity(30, 0.1, 0.02, W, H).astype(np.float32)
    cases = {"empty": np.zeros((H, W), np.uint8)}
    m = np.zeros((H, W), np.uint8); m[3, 5] = m[9, 9] = 1
    cases["two"] = m
    m = np.zeros((H, W), np.uint8); m[17, :] = 1
    cases["row"] = m
    m = np.zeros((H, W), np.uint8); m[:, 40] = 1
    cases["column"] = m
    m = np.zeros((H, W), np.uint8); m[np.arange(H), np.arange(H)] = 1
    cases["diagonal"] = m
    Ms = np.stack(list(cases.values()))
    Ds = np.stack([D] * len(cases))
    fit = lib.road_fit(_dev(Ds), _dev(Ms))
    got = lib.road_fit_dicts(fit)
    for g, M in zip(got, Ms):
        _close_fit(g, oroad.fit_road(D, M), D)
    assert [g["status"] for g in got] == [1, 1, 2, 2, 2]
    # failed fits: windows start at 0, the transformation gives NaN
    lo = lib.road_window(fit, W, H, 24, 1, 2.0, 1.0).cpu().numpy()
    assert not lo.any()
    D2 = lib.disparity_transform(_dev(Ds), fit, 3.0).cpu().numpy()
    assert np.isnan(D2).all()


def _floor_arg(a0, a1, phi, W, H, w, mode, delta):
    """The oracle-side value that floor() sees for each row."""
    cx, cy = (W - 1) / 2, (H - 1) / 2
    v = np.arange(H, dtype=np.float64)
    if mode == 0:
        return a0 + a1 * math.cos(phi) * (v - cy) + 0.5
    ends = [a0 + a1 * (math.cos(phi) * (v - cy) - math.sin(phi) * (x - cx)) for x in (0.0, W - 1.0)]
    return np.minimum(*ends) - delta


@pytest.mark.parametrize("mode,w,delta", [(0, 24, 0.0), (1, 24, 0.0), (1, 16, 3.25), (0, 1, 0.0)])
def test_windows_from_fit_match_oracle(lib, mode, w, delta):
    """Window starts from the device fits equal the oracle's eq. (6) /
    centred windows computed from the oracle's own fits."""
    rng = np.random.default_rng(mode * 10 + w)
    W, H = 320, 240
    maps = []
    for i, (a0, a1, roll) in enumerate([(14.6, 0.0996, 2.0), (30.0, 0.12, -3.0), (5.0, 0.05, 0.5)]):
        D = oroad.road_disparity(a0, a1, math.radians(roll), W, H) + rng.normal(0, 0.3, (H, W))
        maps.append(D.astype(np.float32))
    Ds = np.stack(maps)
    fit = lib.road_fit(_dev(Ds), None, 0.5)
    lo = lib.road_window(fit, W, H, w, mode, delta).cpu().numpy()
    # the same fits used for 4x larger frames: a0 scales by 4, the slopes stay
    lo4 = lib.road_window(fit, 4 * W, 4 * H, w, mode, delta, scale=4.0).cpu().numpy()
    for i in range(len(maps)):
        f = oroad.fit_road(Ds[i], None, 0.5)
        for got, s in ((lo[i], 1), (lo4[i], 4)):
            want = oracle.window_from_road(s * f["a0"], f["a1"], f["phi"], s * W, s * H, w, mode, delta)
            arg = _floor_arg(s * f["a0"], f["a1"], f["phi"], s * W, s * H, w, mode, delta)
            edge = np.abs(arg - np.rint(arg)) < 1e-6
            np.testing.assert_array_equal(got[~edge], want[~edge])
            assert np.all(np.abs(got[edge].astype(int) - want[edge]) <= 1)


def test_transform_matches_oracle_and_in_place(lib):
    ps, D = _sgm_disp(lib, "road320", 4)
    fit = lib.road_fit(_dev(D), _dev(ps.road.astype(np.uint8)))
    f = lib.road_fit_dicts(fit)[0]
    want = oroad.transform(D, f["a0"], f["a1"], f["phi"], 7.5)
    got = lib.disparity_transform(_dev(D), fit, 7.5).cpu().numpy()
    np.testing.assert_allclose(got, want, rtol=2.5e-7, atol=1e-9)
    t = _dev(D)
    lib.disparity_transform(t, fit, 7.5, out=t)
    np.testing.assert_array_equal(t.cpu().numpy(), got)
    # ragged width (scalar path), several maps
    Dr = np.ascontiguousarray(np.stack([D[:, :317], D[::-1, 3:]]))
    fit = lib.road_fit(_dev(Dr), None, 0.5)
    fs = lib.road_fit_dicts(fit)
    got = lib.disparity_transform(_dev(Dr), fit, -2.0).cpu().numpy()
    for i in range(2):
        want = oroad.transform(Dr[i], fs[i]["a0"], fs[i]["a1"], fs[i]["phi"], -2.0)
        np.testing.assert_allclose(got[i], want, rtol=2.5e-7, atol=1e-9)


def test_full_size_batch_of_16(lib):
    """16 maps of 1920 x 1080 in one launch (the learned-window batch shape):
    one map checked against the oracle, every map's count exact and its fit
    on the generated road line; the result is deterministic run to run."""
    import torch
    n, H, W = 16, 1080, 1920
    g = torch.Generator(device="cuda").manual_seed(5)
    v = torch.arange(H, device="cuda", dtype=torch.float64)[:, None] - (H - 1) / 2
    u = torch.arange(W, device="cuda", dtype=torch.float64)[None, :] - (W - 1) / 2
    params = [(40.0 + i, 0.0996, math.radians(-4 + 0.5 * i)) for i in range(n)]
    D = torch.empty((n, H, W), dtype=torch.float32, device="cuda")
    for i, (a0, a1, phi) in enumerate(params):
        noise = torch.randn((H, W), generator=g, device="cuda", dtype=torch.float32) * 0.3
        D[i] = (a0 + a1 * (math.cos(phi) * v - math.sin(phi) * u)).float() + noise
    fit = lib.road_fit(D, None, 0.5)
    fits = lib.road_fit_dicts(fit)
    again = lib.road_fit(D, None, 0.5)
    assert torch.equal(fit, again)
    Dh = D.cpu().numpy()
    counts = (Dh >= 0.5).reshape(n, -1).sum(1)
    for i, (a0, a1, phi) in enumerate(params):
        assert fits[i]["status"] == 0 and fits[i]["count"] == counts[i]
        assert abs(fits[i]["phi"] - phi) < 1e-4 and abs(fits[i]["a1"] - a1) < 1e-4
    _close_fit(fits[9], oroad.fit_road(Dh[9], None, 0.5), Dh[9])
    D2 = lib.disparity_transform(D, fit, 10.0)
    f = fits[9]
    want = oroad.transform(Dh[9], f["a0"], f["a1"], f["phi"], 10.0)
    np.testing.assert_allclose(D2[9].cpu().numpy(), want, rtol=2.5e-7, atol=1e-9)


def _check_fits(lib, fits, tols, D, min_disp, margin):
    """Each fit of a fit-then-refit sequence against the oracle, the oracle
    given the GPU's previous fit as its prior."""
    prior = None
    for k, tol in enumerate((math.inf,) + tuple(tols)):
        f = lib.road_fit_dicts(fits[k])[0]
        _close_fit(f, oroad.fit_road(D, None, min_disp, margin, prior, tol), D)
        prior = (f["a0"], f["a1"], f["phi"])
    return lib.road_fit_dicts(fits[-1])[0]


@pytest.mark.parametrize("windows", ["row", "pixel"])
def test_perspective_pipeline_from_images_alone(lib, windows):
    """The self-contained perspective-transformed path on a 1280x720 road
    pair: every stage equals the oracle on the previous stage's GPU output
    (4x4 reduction and quarter-scale SGM bit-exact, coarse fit and refit,
    row windows or per-pixel windows from the plane at scale 4, windowed
    SGM bit-exact, fit and refits on D1, eq. (13)), and the coarse fit finds
    the scene's own road line."""
    import torch
    from paper_2012_10802_amd.road_pipeline import PerspectiveMatcher
    seed = 5
    sc = synth.scene_for_config("road1280", seed)
    ps = synth.make_pair(sc, seed)
    pm = PerspectiveMatcher(1280, 720, ndisp=128, w=24, census=7, npaths=8, p1=10, p2=120, windows=windows,
                            delta_dt=20.0)
    dint, dsub, d2 = (t[0] for t in pm.match(_dev(ps.left), _dev(ps.right)))
    torch.cuda.synchronize()
    lc, rc = oracle.downsample4(ps.left), oracle.downsample4(ps.right)
    np.testing.assert_array_equal(pm.left_c[0].cpu().numpy(), lc)
    np.testing.assert_array_equal(pm.right_c[0].cpu().numpy(), rc)
    ci, cs = oracle.sgm(lc, rc, 7, 32, 8, 10, 120)
    np.testing.assert_array_equal(pm.coarse_int[0].cpu().numpy().view(np.uint16), ci)
    np.testing.assert_allclose(pm.coarse_sub[0].cpu().numpy(), cs, rtol=0, atol=1e-4)
    cmap = pm.coarse_sub[0].cpu().numpy()
    cf = _check_fits(lib, pm.coarse_fits, pm.coarse_tols, cmap, 0.5, 4.0)
    a0, a1, phi = ps.road_params
    assert abs(cf["phi"] - phi) < math.radians(0.2) and abs(4 * cf["a0"] - a0) < 1.0
    if windows == "row":
        want = oracle.window_from_road(4 * cf["a0"], cf["a1"], cf["phi"], 1280, 720, 24, 0)
        arg = _floor_arg(4 * cf["a0"], cf["a1"], cf["phi"], 1280, 720, 24, 0, 0.0)
        edge = np.abs(arg - np.rint(arg)) < 1e-6
        d_lo = pm.d_lo[0].cpu().numpy()
        np.testing.assert_array_equal(d_lo[~edge], want[~edge])
        oi, osub = oracle.sgm(ps.left, ps.right, 7, 24, 8, 10, 120, d_lo)
    else:
        lo = pm.lo[0].cpu().numpy()
        want = oroad.window_map(cf["a0"], cf["a1"], cf["phi"], 1280, 720, 16, 4.0)
        f = oroad.road_disparity(4 * cf["a0"], cf["a1"], cf["phi"], 1280, 720) + 0.5
        edge = np.abs(f - np.rint(f)) < 1e-6
        np.testing.assert_array_equal(lo[~edge], want[~edge])
        oi, osub = oracle.sgm_win(ps.left, ps.right, 7, 16, 8, 10, 120, lo)
        # the windows hold the scene's road: ground truth inside them on the road
        road = ps.road & ~ps.pothole
        inside = (ps.gt >= lo) & (ps.gt <= lo + 15)
        assert inside[road].mean() > 0.999
    np.testing.assert_array_equal(dint.cpu().numpy().view(np.uint16), oi)
    np.testing.assert_allclose(dsub.cpu().numpy(), osub, rtol=0, atol=1e-4)
    D1 = dsub.cpu().numpy()
    f = _check_fits(lib, pm.fits, pm.fine_tols, D1, 2.0, 16.0)
    np.testing.assert_allclose(d2.cpu().numpy(), oroad.transform(D1, f["a0"], f["a1"], f["phi"], 20.0),
                               rtol=2.5e-7, atol=1e-9)


def test_road_mask_matches_oracle(lib):
    """The road region from device fits equals the oracle's from the same
    (a0, a1, phi), except on pixels whose road disparity lies within 1e-9 of
    f_min (the two evaluate the line in another order); failed fits give an
    empty mask."""
    rng = np.random.default_rng(12)
    W, H = 321, 200
    Ds = []
    for a0, a1, roll in ((14.0, 0.1, 2.0), (20.0, 0.12, -3.0)):
        D = oroad.road_disparity(a0, a1, math.radians(roll), W, H) + rng.normal(0, 0.3, (H, W))
        D[D < 0.5] = 0.0
        Ds.append(D.astype(np.float32))
    Ds = np.stack(Ds + [np.zeros((H, W), np.float32)])
    Ds[1, 5, 7] = np.nan
    fit = lib.road_fit(_dev(Ds), None, 0.5, 4.0)
    fs = lib.road_fit_dicts(fit)
    assert [f["status"] for f in fs] == [0, 0, 1]
    got = lib.road_mask(_dev(Ds), fit, 2.0, 4.0).cpu().numpy()
    for i in range(2):
        f = fs[i]
        want = oroad.road_mask(Ds[i], f["a0"], f["a1"], f["phi"], 2.0, 4.0)
        edge = np.abs(oroad.road_disparity(f["a0"], f["a1"], f["phi"], W, H) - 2.0) < 1e-9
        np.testing.assert_array_equal(got[i][~edge], want[~edge])
        assert 0.2 < want.mean() < 0.95
    assert not got[2].any()


def test_refit_over_the_first_fits_road(lib):
    """Refits with a prior fit (in place, prior = fit) select exactly the
    oracle's pixels within tol of the prior road line."""
    ps, D = _sgm_disp(lib, "road640", 9)
    fit = lib.road_fit(_dev(D), None, 0.5, 4.0)
    prior = lib.road_fit_dicts(fit)[0]
    for tol in (2.0, 1.0, 0.5):
        lib.road_fit(_dev(D), None, 0.5, 4.0, prior=fit, tol=tol, fit=fit)
        got = lib.road_fit_dicts(fit)[0]
        want = oroad.fit_road(D, None, 0.5, 4.0, (prior["a0"], prior["a1"], prior["phi"]), tol)
        _close_fit(got, want, D)
        prior = got
    a0, a1, phi = ps.road_params
    assert abs(prior["a1"] - a1) < 2e-3 and abs(prior["phi"] - phi) < 2e-3


def test_window_map_matches_oracle(lib):
    """Per-pixel windows from device fits (scale 1 and 4) equal the oracle's
    from the same parameters, except where f + 1/2 lies within 1e-6 of an
    integer; a failed fit gives zeros."""
    rng = np.random.default_rng(21)
    W, H = 160, 120
    Ds = [(oroad.road_disparity(a0, a1, math.radians(r), W, H) + rng.normal(0, 0.2, (H, W))).astype(np.float32)
          for a0, a1, r in ((10.0, 0.1, 2.5), (20.0, 0.15, -1.0))]
    Ds = np.stack(Ds + [np.zeros((H, W), np.float32)])
    fit = lib.road_fit(_dev(Ds), None, 0.5)
    fs = lib.road_fit_dicts(fit)
    for s_ in (1.0, 4.0):
        Wf, Hf = int(W * s_), int(H * s_)
        lo = lib.road_window_map(fit, Wf, Hf, 16, scale=s_).cpu().numpy()
        for i in range(2):
            f = fs[i]
            want = oroad.window_map(f["a0"], f["a1"], f["phi"], Wf, Hf, 16, s_)
            x = oroad.road_disparity(s_ * f["a0"], f["a1"], f["phi"], Wf, Hf) + 0.5
            edge = np.abs(x - np.rint(x)) < 1e-6
            np.testing.assert_array_equal(lo[i][~edge], want[~edge])
        assert not lo[2].any()


def test_perspective_pipeline_batch_equals_single_frames(lib):
    """A batch of three frames gives, frame by frame, what batches of one
    give (per-pixel windows)."""
    import torch
    from paper_2012_10802_amd.road_pipeline import PerspectiveMatcher
    ps = [synth.make_pair(synth.scene_for_config("road640", s), s) for s in (41, 42, 43)]
    L = _dev(np.stack([p.left for p in ps]))
    R = _dev(np.stack([p.right for p in ps]))
    pm3 = PerspectiveMatcher(640, 480, batch=3, ndisp=64)
    out3 = [t.clone() for t in pm3.match(L, R)]
    pm1 = PerspectiveMatcher(640, 480, batch=1, ndisp=64)
    for i in range(3):
        out1 = pm1.match(L[i], R[i])
        for a, b in zip(out3, out1):
            assert torch.equal(a[i], b[0])
        assert torch.equal(pm3.lo[i], pm1.lo[0])


def _oracle_curve(D, phis, mask=None, min_disp=-math.inf, margin=-math.inf, prior=None, tol=math.inf):
    u, v, d = oroad.select(D, mask, min_disp, margin, prior, tol)
    out = []
    for p in phis:
        if len(d) < 2 or np.linalg.matrix_rank(oroad.T_matrix(u, v, p)) < 2:
            out.append(math.nan)
        else:
            out.append(oroad.e0min(u, v, d, p))
    return np.array(out)


def _close_curve(got, want, D):
    sdd = float(np.nansum(np.where(np.isfinite(D), D.astype(np.float64), 0.0) ** 2))
    np.testing.assert_array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    np.testing.assert_allclose(got[ok], want[ok], rtol=1e-6, atol=1e-10 * sdd + 1e-12)


def test_energy_curve_matches_oracle(lib):
    """E0min(phi) of eq. (12) (Fig. 3) at 181 roll angles over a half turn:
    the hand-worked map, and SGM output of a generated road pair with the
    selections a pipeline uses (floor, margin, a refit's prior and tol)."""
    import torch
    phis = np.linspace(-math.pi / 2, math.pi / 2, 181)[1:]
    ph = _dev(phis)
    with open(os.path.join(GOLD, "hand_road3x3.json")) as f:
        D = np.array(json.load(f)["disp"], np.float32)
    got = lib.road_energy(_dev(D), ph).cpu().numpy()[0]
    _close_curve(got, _oracle_curve(D, phis), D)
    ps, D = _sgm_disp(lib, "road640", 7)
    got = lib.road_energy(_dev(D), ph, _dev(ps.road.astype(np.uint8))).cpu().numpy()[0]
    _close_curve(got, _oracle_curve(D, phis, ps.road), D)
    got = lib.road_energy(_dev(D), ph, None, 0.5, 4.0).cpu().numpy()[0]
    _close_curve(got, _oracle_curve(D, phis, None, 0.5, 4.0), D)
    fit = lib.road_fit(_dev(D), None, 0.5, 4.0)
    f = lib.road_fit_dicts(fit)[0]
    got = lib.road_energy(_dev(D), ph, None, 0.5, 4.0, prior=fit, tol=2.0).cpu().numpy()[0]
    _close_curve(got, _oracle_curve(D, phis, None, 0.5, 4.0, (f["a0"], f["a1"], f["phi"]), 2.0), D)
    torch.cuda.synchronize()


def test_energy_curve_minimum_is_the_fit(lib):
    """The curve's value at the fitted roll equals the fit's E0min, and no
    angle of a fine grid lies below it: the closed form finds the minimum
    of the curve that Sec. II-C searches."""
    ps, D = _sgm_disp(lib, "road320", 2)
    d = _dev(D)
    m = _dev(ps.road.astype(np.uint8))
    f = lib.road_fit_dicts(lib.road_fit(d, m))[0]
    assert f["status"] == 0
    phis = np.concatenate([[f["phi"]], f["phi"] + np.linspace(-0.05, 0.05, 2001), np.linspace(-1.5, 1.5, 301)])
    e = lib.road_energy(d, _dev(phis), m).cpu().numpy()[0]
    sdd = float(np.sum(D[ps.road].astype(np.float64) ** 2))
    assert e[0] == pytest.approx(f["e0min"], rel=1e-6, abs=1e-10 * sdd)
    assert e.min() >= e[0] - 1e-10 * sdd
    assert np.argmin(e[1:2002]) in range(995, 1006)  # the grid's minimum sits next to the fitted phi


def test_energy_curve_degenerate_maps(lib):
    """A one-row map: y = v is constant at phi = 0 (NaN) but not at other
    angles; a one-pixel selection: NaN everywhere; both in one batch with a
    regular map."""
    import torch
    rng = np.random.default_rng(5)
    W = 40
    D = np.stack([np.full((3, W), np.nan, np.float32) for _ in range(3)])
    D[0, 1] = 5.0 + 0.1 * np.arange(W) + rng.normal(0, 0.05, W)  # one row
    D[1, 2, 7] = 3.0  # one pixel
    D[2] = 4.0 + 0.2 * np.arange(3)[:, None] + 0.05 * np.arange(W)[None, :]
    phis = np.array([0.0, 0.3, -1.2])
    e = lib.road_energy(_dev(D), _dev(phis)).cpu().numpy()
    assert math.isnan(e[0, 0]) and np.isfinite(e[0, 1:]).all()
    assert np.isnan(e[1]).all()
    assert np.isfinite(e[2]).all()
    for i in range(3):
        _close_curve(e[i], _oracle_curve(D[i], phis), D[i])
    torch.cuda.synchronize()
