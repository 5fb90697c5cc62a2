"""Pins of the CPU oracle to facts fixed outside it.

The paper prints no worked example, so each pin comes from the equations
themselves: hand-worked fixtures (tests/golden), brute-force enumeration of
the path energy, closed-form special cases, invariants and exact recovery of
known integer disparities.  Each is chosen so that a plausible slip in the
oracle (a dropped penalty, a reversed path, a swapped image, a wrong census
comparison, a wrong tie-break or parabola sign) fails at least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_2012_10802_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------------------
# hand-worked fixtures


def test_hand_scanline_paths_sum_and_selection():
    """eq. (8) with the -min term, eq. (9) argmin and the parabola, by hand."""
    g = _gold("hand_scanline.json")
    c = np.array(g["cost"], np.uint8)
    np.testing.assert_array_equal(oracle.path(c, 0, g["p1"], g["p2"]), g["L_path0"])
    np.testing.assert_array_equal(oracle.path(c, 1, g["p1"], g["p2"]), g["L_path1"])
    S = oracle.sum_paths(c, 4, g["p1"], g["p2"])
    np.testing.assert_array_equal(S, g["S4"])
    dint, dsub = oracle.wta(S)
    np.testing.assert_array_equal(dint, g["dint"])
    want = [np.float32(k) + np.float32(n) / np.float32(d)
            for k, (n, d) in zip(g["dint"][0], g["dsub_num_den"])]
    np.testing.assert_array_equal(dsub[0], np.array(want, np.float32))


def test_hand_census3():
    g = _gold("hand_census3.json")
    codes = oracle.census(np.array(g["image"], np.uint8), 3)
    for key, val in g["codes"].items():
        u, v = map(int, key.split(","))
        assert int(codes[v, u]) == val, key


# ---------------------------------------------------------------------------
# brute force: the path DP is a min-sum over disparity sequences


def _pen(a, b, p1, p2):
    d = abs(a - b)
    return 0 if d == 0 else (p1 if d == 1 else p2)


def _path_pixels(u, v, du, dv, W, H):
    """Pixels of the path through (u, v) along r = (du, dv), start first."""
    pix = [(u, v)]
    while True:
        qu, qv = pix[-1][0] - du, pix[-1][1] - dv
        if not (0 <= qu < W and 0 <= qv < H):
            break
        pix.append((qu, qv))
    return pix[::-1]


def _brute_energy(c, pix, k, p1, p2):
    """min over disparity sequences ending at k of sum C + sum penalties."""
    w = c.shape[2]
    best = None
    for seq in itertools.product(range(w), repeat=len(pix) - 1):
        seq = seq + (k,)
        e = sum(int(c[v, u, d]) for (u, v), d in zip(pix, seq))
        e += sum(_pen(seq[i - 1], seq[i], p1, p2) for i in range(1, len(seq)))
        best = e if best is None or e < best else best
    return best


@pytest.mark.parametrize("r", range(8))
def test_path_equals_bruteforce_min_sum(r):
    """Un-normalised L_r(p,k) is the best path energy ending at (p,k) when
    P1 <= P2; the normalised form subtracts the previous pixel's minimum."""
    rng = np.random.default_rng(100 + r)
    H, W, w = 3, 4, 3
    c = rng.integers(0, 25, size=(H, W, w), dtype=np.uint8)
    p1, p2 = 3, 7
    du, dv = oracle.PATHS[r]
    L = oracle.path(c, r, p1, p2)
    U = oracle.path_raw(c, r, p1, p2)
    for v in range(H):
        for u in range(W):
            pix = _path_pixels(u, v, du, dv, W, H)
            ub = [_brute_energy(c, pix, k, p1, p2) for k in range(w)]
            assert list(U[v, u]) == ub
            if len(pix) == 1:
                assert list(L[v, u]) == list(c[v, u])
            else:
                qu, qv = pix[-2]
                mq = min(_brute_energy(c, pix[:-1], k, p1, p2) for k in range(w))
                assert list(L[v, u]) == [x - mq for x in ub]


def test_bruteforce_wider_window_longer_path():
    rng = np.random.default_rng(7)
    H, W, w = 1, 6, 4
    c = rng.integers(0, 50, size=(H, W, w), dtype=np.uint8)
    p1, p2 = 4, 11
    for r in (0, 1):
        du, dv = oracle.PATHS[r]
        U = oracle.path_raw(c, r, p1, p2)
        for u in range(W):
            pix = _path_pixels(u, 0, du, dv, W, H)
            assert list(U[0, u]) == [_brute_energy(c, pix, k, p1, p2) for k in range(w)]


# ---------------------------------------------------------------------------
# closed-form special cases


def _rand_cost(seed, H=17, W=23, w=9, hi=49):
    return np.random.default_rng(seed).integers(0, hi, size=(H, W, w), dtype=np.uint8)


@pytest.mark.parametrize("npaths", [4, 8])
def test_zero_penalties_reduce_to_local_wta(npaths):
    """P1 = P2 = 0: every L_r = C, so S = R*C and k* = argmin_k C."""
    c = _rand_cost(1)
    for r in range(npaths):
        np.testing.assert_array_equal(oracle.path(c, r, 0, 0), c)
    S = oracle.sum_paths(c, npaths, 0, 0)
    np.testing.assert_array_equal(S, npaths * c.astype(np.uint32))
    dint, _ = oracle.wta(S)
    np.testing.assert_array_equal(dint, np.argmin(c, axis=2))


def test_single_disparity_window():
    c = _rand_cost(2, w=1)
    S = oracle.sum_paths(c, 8, 10, 120)
    np.testing.assert_array_equal(S, 8 * c.astype(np.uint32))
    dint, dsub = oracle.wta(S)
    assert (dint == 0).all() and (dsub == 0).all()


def test_wta_ties_go_to_smallest_disparity():
    S = np.zeros((2, 3, 5), np.uint32) + 9
    S[0, 0, [1, 3]] = 2
    S[1, 2, [0, 4]] = 1
    S[0, 1, [2, 3]] = 0
    dint, dsub = oracle.wta(S)
    assert dint[0, 0] == 1 and dint[1, 2] == 0 and dint[0, 1] == 2
    assert dint[1, 0] == 0  # all equal
    # k*=2 with S(3) == S(2): the vertex sits half-way, delta = +1/2
    assert dsub[0, 1] == np.float32(2.5)


def test_parabola_vertex_is_recovered():
    """S sampled from an integer parabola A(k-k0)^2 - B(k-k0) + c0 with
    |B| < A has its minimum at k0 and its vertex at k0 + B/(2A)."""
    w = 16
    cases = [(4, 2, 7), (4, -2, 7), (8, 3, 5), (2, 0, 9), (10, 9, 1), (6, -5, 14)]
    S = np.zeros((1, len(cases), w), np.uint32)
    for i, (A, B, k0) in enumerate(cases):
        k = np.arange(w) - k0
        S[0, i] = A * k * k - B * k + 100
    dint, dsub = oracle.wta(S)
    for i, (A, B, k0) in enumerate(cases):
        assert dint[0, i] == k0
        assert dsub[0, i] == np.float32(k0) + np.float32(B) / np.float32(2 * A)


# ---------------------------------------------------------------------------
# invariants


@pytest.fixture(scope="module")
def road320():
    p = synth.make_pair(synth.scene_for_config("road320", 11), 11)
    cl = oracle.census(p.left, 5)
    cr = oracle.census(p.right, 5)
    return p, oracle.cost(cl, cr, 5, 32)


def test_aggregation_bounded_by_p2(road320):
    """0 <= L_r - C <= P2 for every path, pixel and disparity."""
    _, c = road320
    ci = c.astype(np.int32)
    for r in range(8):
        d = oracle.path(c, r, 10, 120).astype(np.int32) - ci
        assert d.min() >= 0 and d.max() <= 120


def test_normalised_and_literal_forms_select_the_same(road320):
    """Dropping the -min term shifts each L_r(p,.) by a constant: the
    argmin and sub-pixel offset of S are unchanged."""
    _, c = road320
    c = c[:80, :120]
    S = oracle.sum_paths(c, 8, 10, 120)
    U = sum(oracle.path_raw(c, r, 10, 120) for r in range(8))
    shift = U - S.astype(np.int64)
    assert (shift == shift[:, :, :1]).all()
    a = oracle.wta(S)
    b = oracle.wta((U - U.min(axis=2, keepdims=True)).astype(np.uint32))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_vertical_flip_equivariance(road320):
    p, _ = road320
    lo = np.random.default_rng(3).integers(0, 6, size=p.left.shape[0]).astype(np.int32)
    a = oracle.sgm(p.left, p.right, 5, 24, 8, 10, 120, lo)
    b = oracle.sgm(p.left[::-1], p.right[::-1], 5, 24, 8, 10, 120, lo[::-1])
    np.testing.assert_array_equal(a[0], b[0][::-1])
    np.testing.assert_array_equal(a[1], b[1][::-1])


# ---------------------------------------------------------------------------
# census


def test_census_constant_and_monotone_invariance():
    rng = np.random.default_rng(5)
    assert (oracle.census(np.full((9, 11), 77, np.uint8), 7) == 0).all()
    img = rng.integers(0, 120, size=(20, 31), dtype=np.uint8)
    lut = np.cumsum(rng.integers(1, 3, size=256))  # strictly increasing
    assert lut[119] < 256
    mapped = lut[img].astype(np.uint8)
    for n in (3, 5, 7):
        np.testing.assert_array_equal(oracle.census(img, n), oracle.census(mapped, n))


def test_census_bit_count():
    rng = np.random.default_rng(6)
    img = rng.integers(0, 256, size=(16, 16), dtype=np.uint8)
    for n in (5, 7):
        codes = oracle.census(img, n)
        assert int(codes.max()) < (1 << (n * n - 1))
        # the strict global maximum pixel of a window has every other bit set
    flat = np.zeros((7, 7), np.uint8)
    flat[3, 3] = 200
    assert int(oracle.census(flat, 7)[3, 3]) == (1 << 48) - 1
    assert int(oracle.census(flat, 5)[3, 3]) == (1 << 24) - 1


# ---------------------------------------------------------------------------
# cost and per-row windows


def test_cost_identity_and_out_of_image():
    rng = np.random.default_rng(8)
    img = rng.integers(0, 256, size=(12, 40), dtype=np.uint8)
    cl = oracle.census(img, 7)
    c = oracle.cost(cl, cl, 7, 6)
    assert (c[:, :, 0] == 0).all()
    for k in range(6):
        assert (c[:, :k, k] == 48).all()  # right column u - k < 0


def test_window_start_shifts_the_cost_range():
    """A window [c, c+w) on every row is the slice [c, c+w) of the plain
    cost over [0, c+w)."""
    p = synth.make_pair(synth.RoadScene(96, 40, focal=120.0, roll_deg=1.0), 4)
    cl, cr = oracle.census(p.left, 7), oracle.census(p.right, 7)
    full = oracle.cost(cl, cr, 7, 30)
    for c0 in (0, 3, 11):
        win = oracle.cost(cl, cr, 7, 12, np.full(40, c0, np.int32))
        np.testing.assert_array_equal(win, full[:, :, c0:c0 + 12])
    lo = np.arange(40, dtype=np.int32) % 7
    win = oracle.cost(cl, cr, 7, 12, lo)
    for v in range(40):
        np.testing.assert_array_equal(win[v], full[v, :, lo[v]:lo[v] + 12])


def test_zero_window_start_is_plain_sgm(road320):
    p, _ = road320
    a = oracle.sgm(p.left, p.right, 5, 32, 4, 10, 120)
    b = oracle.sgm(p.left, p.right, 5, 32, 4, 10, 120, np.zeros(240, np.int32))
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_window_from_road_closed_forms():
    W, H = 640, 480
    cx, cy = (W - 1) / 2, (H - 1) / 2
    # no roll, centred window of width 24 around a0 + a1 (v - cy)
    d = oracle.window_from_road(20.0, 0.1, 0.0, W, H, 24, mode=0)
    want = [max(0, math.floor(20.0 + 0.1 * (v - cy) + 0.5) - 12) for v in range(H)]
    assert list(d) == want
    # eq. (6): a linear function of x is smallest at an end of the row
    a0, a1, phi, delta = 30.0, 0.12, math.radians(3.0), 4.0
    d = oracle.window_from_road(a0, a1, phi, W, H, 24, mode=1, delta=delta)
    for v in range(H):
        ends = [a0 + a1 * (math.cos(phi) * (v - cy) - math.sin(phi) * (x - cx)) - delta
                for x in (0, W - 1)]
        assert d[v] == max(0, math.floor(min(ends)))


# ---------------------------------------------------------------------------
# exact recovery of integer disparities on textured fronto-parallel planes


def _shifted_pair(W, H, d_of_row, seed):
    rng = np.random.default_rng(seed)
    L = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    R = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    for v in range(H):
        d = d_of_row[v]
        R[v, : W - d] = L[v, d:]  # right column x shows left column x + d
    return L, R


def test_exact_recovery_integer_plane():
    W, H, d0, n = 160, 48, 9, 7
    L, R = _shifted_pair(W, H, [d0] * H, 21)
    dint, dsub = oracle.sgm(L, R, n, 32, 8, 10, 120)
    band = dint[:, d0 + 3 + 16: W - 3 - 16]
    assert (band == d0).all()
    assert (np.abs(dsub[:, d0 + 19: W - 19] - d0) <= 0.5).all()


def test_exact_recovery_staircase():
    W, H, n = 160, 96, 5
    steps = [4, 12, 20]
    rows = [steps[v * 3 // H] for v in range(H)]
    L, R = _shifted_pair(W, H, rows, 22)
    dint, _ = oracle.sgm(L, R, n, 32, 8, 10, 120)
    for i, d0 in enumerate(steps):
        v0, v1 = i * H // 3 + 16, (i + 1) * H // 3 - 16
        assert (dint[v0:v1, d0 + 2 + 16: W - 2 - 16] == d0).all()


def test_recovery_with_row_windows():
    """The same plane seen through row windows that contain d0.  Smoothness
    acts on the window index (the disparity of the transformed pair, D0), so
    the window start is held constant over blocks of rows and recovery is
    checked away from the block edge."""
    W, H, d0 = 160, 80, 23
    L, R = _shifted_pair(W, H, [d0] * H, 23)
    lo = np.where(np.arange(H) < H // 2, d0 - 5, d0 - 9).astype(np.int32)
    dint, _ = oracle.sgm(L, R, 7, 12, 8, 10, 120, lo)
    rows = np.r_[0:H // 2 - 16, H // 2 + 16:H]
    assert (dint[rows, d0 + 19: W - 19] == d0).all()


# ---------------------------------------------------------------------------
# the generator agrees with the road model of eq. (3)


def test_generator_ground_truth_is_the_road_model():
    s = synth.RoadScene(320, 240, focal=300.0, roll_deg=2.0)
    p = synth.make_pair(s, 31)
    a0, a1, phi = p.road_params
    vv, uu = np.mgrid[0:240, 0:320].astype(np.float64)
    plane = p.road & ~p.pothole
    f = a0 + a1 * (np.cos(phi) * (vv - s.cy) - np.sin(phi) * (uu - s.cx))
    assert np.abs(p.gt[plane] - f[plane]).max() < 1e-9
    # eq. (11) at the true roll recovers a, and the residual of eq. (12) vanishes
    d = p.gt[plane]
    T = np.stack([np.ones_like(d), np.cos(phi) * (vv - s.cy)[plane]
                  - np.sin(phi) * (uu - s.cx)[plane]], 1)
    a, res, *_ = np.linalg.lstsq(T, d, rcond=None)
    assert abs(a[0] - a0) < 1e-9 and abs(a[1] - a1) < 1e-12
    assert float(np.sum((d - T @ a) ** 2)) < 1e-12
    # potholes are deeper: lower disparity than the plane
    assert (p.gt[p.pothole] < f[p.pothole]).all()


def test_torch_renderer_matches_generator():
    """The torch renderer (used for training data) draws the same scene:
    identical clean images, road mask and ground truth."""
    import dataclasses
    s = dataclasses.replace(synth.scene_for_config("road640", 4), noise_sigma=0.0)
    p = synth.make_pair(s, 4)
    left, right, gt, road = synth.make_pair_torch(s, 4, device="cpu", noise=False)
    np.testing.assert_array_equal(left.numpy(), p.left)
    np.testing.assert_array_equal(right.numpy(), p.right)
    np.testing.assert_array_equal(road.numpy(), p.road)
    assert np.abs(gt.numpy() - p.gt).max() < 1e-5
    noisy_l, _, _, _ = synth.make_pair_torch(dataclasses.replace(s, noise_sigma=2.0), 4, device="cpu")
    diff = noisy_l.numpy().astype(float) - p.left
    assert 1.5 < diff.std() < 2.5


# ---------------------------------------------------------------------------
# per-pixel windows in absolute disparity (learned-window form)


def _brute_energy_win(c, lo, pix, d_end, p1, p2):
    """min over absolute-disparity sequences, d_i in the window of pixel i,
    ending at d_end, of sum C + sum penalties."""
    w = c.shape[2]
    choices = [range(lo[v, u], lo[v, u] + w) for (u, v) in pix[:-1]]
    best = None
    for seq in itertools.product(*choices):
        seq = seq + (d_end,)
        e = sum(int(c[v, u, d - lo[v, u]]) for (u, v), d in zip(pix, seq))
        e += sum(_pen(seq[i - 1], seq[i], p1, p2) for i in range(1, len(seq)))
        best = e if best is None or e < best else best
    return best


@pytest.mark.parametrize("r", range(8))
def test_window_path_equals_bruteforce(r):
    rng = np.random.default_rng(300 + r)
    H, W, w = 3, 4, 3
    c = rng.integers(0, 25, size=(H, W, w), dtype=np.uint8)
    lo = rng.integers(0, 4, size=(H, W)).astype(np.int32)
    p1, p2 = 3, 7
    du, dv = oracle.PATHS[r]
    L = oracle.path_win(c, lo, r, p1, p2)
    for v in range(H):
        for u in range(W):
            pix = _path_pixels(u, v, du, dv, W, H)
            ub = [_brute_energy_win(c, lo, pix, lo[v, u] + j, p1, p2) for j in range(w)]
            if len(pix) == 1:
                assert list(L[v, u]) == list(c[v, u])
            else:
                qu, qv = pix[-2]
                mq = min(_brute_energy_win(c, lo, pix[:-1], lo[qv, qu] + j, p1, p2) for j in range(w))
                assert list(L[v, u]) == [x - mq for x in ub]


def test_window_constant_start_is_row_window_sgm(road320):
    p, _ = road320
    for c0 in (0, 5):
        lo = np.full(p.left.shape, c0, np.int32)
        a = oracle.sgm_win(p.left, p.right, 5, 16, 8, 10, 120, lo)
        b = oracle.sgm(p.left, p.right, 5, 16, 8, 10, 120, np.full(240, c0, np.int32))
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])


def test_window_cost_is_slice_of_full_cost():
    p = synth.make_pair(synth.RoadScene(96, 40, focal=120.0, roll_deg=1.0), 8)
    cl, cr = oracle.census(p.left, 7), oracle.census(p.right, 7)
    full = oracle.cost(cl, cr, 7, 40)
    lo = np.random.default_rng(1).integers(0, 25, size=(40, 96)).astype(np.int32)
    win = oracle.cost_win(cl, cr, 7, 16, lo)
    for v in range(40):
        for u in range(96):
            np.testing.assert_array_equal(win[v, u], full[v, u, lo[v, u]:lo[v, u] + 16])


def test_window_exact_recovery_with_random_windows():
    """Absolute-disparity smoothness: a plane at integer d0 is recovered
    through per-pixel windows that contain d0 at random positions."""
    W, H, d0 = 160, 48, 21
    L, R = _shifted_pair(W, H, [d0] * H, 24)
    lo = (d0 - np.random.default_rng(2).integers(0, 16, size=(H, W))).astype(np.int32)
    dint, dsub = oracle.sgm_win(L, R, 7, 16, 8, 10, 120, lo)
    band = dint[:, d0 + 3 + 16: W - 3 - 16]
    assert (band == d0).all()


def test_downsample4_closed_forms():
    img = np.arange(16, dtype=np.uint8).reshape(4, 4)
    assert oracle.downsample4(img)[0, 0] == (120 + 8) // 16
    assert (oracle.downsample4(np.full((13, 9), 200, np.uint8)) == 200).all()
    assert oracle.downsample4(np.full((13, 9), 200, np.uint8)).shape == (3, 2)
    rng = np.random.default_rng(4)
    big = rng.integers(0, 256, size=(8, 12), dtype=np.uint8)
    want = (big.reshape(2, 4, 3, 4).astype(int).sum(axis=(1, 3)) + 8) // 16
    np.testing.assert_array_equal(oracle.downsample4(big), want)
