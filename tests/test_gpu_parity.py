"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Integer outputs (census codes, costs, per-path L_r, the sum S and the
integer disparity) must match bit for bit.  The sub-pixel disparity is one
IEEE fp32 division and one addition on exact integers on both sides, so it
is expected to match exactly too; the bar written here is the stated
1e-4 px.
"""
import numpy as np
import pytest

import oracle
from paper_2012_10802_amd import synth

pytestmark = pytest.mark.gpu

SUB_TOL = 1e-4


@pytest.fixture(scope="module")
def lib():
    import torch
    from paper_2012_10802_amd import sgm
    assert torch.cuda.is_available()
    return sgm


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _np_u16(t):
    return t.cpu().numpy().view(np.uint16)


def _rand_pair(W, H, seed, shift=5):
    rng = np.random.default_rng(seed)
    L = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    R = np.roll(L, -shift, axis=1)
    R = np.clip(R.astype(int) + rng.integers(-3, 4, size=(H, W)), 0, 255).astype(np.uint8)
    return L, R


# (W, H, census, w, npaths): ragged tails in every dimension, windows that
# do not fill a lane row, a single disparity, the widest window
SHAPES = [
    (37, 11, 5, 32, 4),
    (70, 23, 7, 24, 8),
    (133, 41, 7, 128, 8),
    (50, 19, 3, 64, 8),
    (17, 64, 7, 192, 8),
    (40, 9, 5, 256, 8),
    (29, 13, 7, 100, 8),
    (23, 7, 5, 1, 4),
    (1, 30, 5, 16, 8),
    (45, 1, 7, 20, 8),
    # cost tiles staged through LDS (w >= 64): a one-pixel column, a full
    # tile, a tile plus one pixel
    (1, 9, 7, 64, 8),
    (64, 5, 5, 128, 4),
    (65, 3, 7, 192, 4),
]


@pytest.mark.parametrize("n", [3, 5, 7])
def test_census_matches_oracle(lib, n):
    import torch
    for W, H in [(64, 4), (131, 37), (5, 3)]:
        img = np.random.default_rng(W * H + n).integers(0, 256, size=(H, W), dtype=np.uint8)
        m = lib.Matcher(W, H, census=n, ndisp=8, npaths=4)
        codes = m.census(_dev(img))
        torch.cuda.synchronize()
        got = codes.cpu().numpy().view(np.uint64)
        np.testing.assert_array_equal(got, oracle.census(img, n))


def test_census_with_pitch(lib):
    import torch
    W, H, pitch = 50, 20, 64
    buf = np.random.default_rng(3).integers(0, 256, size=(H, pitch), dtype=np.uint8)
    m = lib.Matcher(W, H, census=7, ndisp=8, npaths=4)
    got = m.census(_dev(buf)).cpu().numpy().view(np.uint64)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got, oracle.census(buf[:, :W], 7))


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_cost_and_paths_match_oracle(lib, shape):
    import torch
    W, H, n, w, R = shape
    L, Rimg = _rand_pair(W, H, 11 + W)
    rng = np.random.default_rng(W + H)
    d_lo = rng.integers(0, 6, size=H).astype(np.int32)
    m = lib.Matcher(W, H, census=n, ndisp=w, npaths=R, p1=10, p2=120)
    cost = m.cost(_dev(L), _dev(Rimg), d_lo=_dev(d_lo))
    torch.cuda.synchronize()
    want_c = oracle.cost(oracle.census(L, n), oracle.census(Rimg, n), n, w, d_lo)
    np.testing.assert_array_equal(cost.cpu().numpy(), want_c)
    for r in range(8):
        Lr = m.aggregate_path(cost, r)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(_np_u16(Lr), oracle.path(want_c, r, 10, 120), err_msg="path %d" % r)
    S = m.aggregate(cost)
    torch.cuda.synchronize()
    want_S = oracle.sum_paths(want_c, R, 10, 120)
    np.testing.assert_array_equal(_np_u16(S).astype(np.uint32), want_S)
    dint, dsub = m.wta(S, d_lo=_dev(d_lo))
    torch.cuda.synchronize()
    wi, ws = oracle.wta(want_S, d_lo)
    np.testing.assert_array_equal(_np_u16(dint), wi)
    assert np.abs(dsub.cpu().numpy() - ws).max() <= SUB_TOL
    np.testing.assert_array_equal(dsub.cpu().numpy(), ws)
    dint2, dsub2 = m.aggregate_wta(cost, d_lo=_dev(d_lo))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np_u16(dint2), wi)
    np.testing.assert_array_equal(dsub2.cpu().numpy(), ws)


@pytest.mark.parametrize("p1,p2", [(0, 0), (3, 7), (10, 120), (1, 200), (60, 60)])
def test_penalty_range(lib, p1, p2):
    """Penalties including P1 = P2 = 0 and uint16 per-path storage (Cmax + P2 > 255)."""
    import torch
    W, H, n, w = 61, 27, 7, 48
    L, Rimg = _rand_pair(W, H, 5)
    m = lib.Matcher(W, H, census=n, ndisp=w, npaths=8, p1=p1, p2=p2)
    cost = m.cost(_dev(L), _dev(Rimg))
    S = m.aggregate(cost)
    dint, dsub = m.aggregate_wta(cost)
    torch.cuda.synchronize()
    c = cost.cpu().numpy()
    want_S = oracle.sum_paths(c, 8, p1, p2)
    np.testing.assert_array_equal(_np_u16(S).astype(np.uint32), want_S)
    wi, ws = oracle.wta(want_S)
    np.testing.assert_array_equal(_np_u16(dint), wi)
    np.testing.assert_array_equal(dsub.cpu().numpy(), ws)


def test_wta_on_oracle_sum_with_ties(lib):
    """Selection on a given S: ties, plateaus and edge minima."""
    import torch
    W, H, w = 33, 5, 40
    rng = np.random.default_rng(9)
    S = rng.integers(0, 6, size=(H, W, w)).astype(np.uint32)  # many ties
    S[0, 0] = 3
    S[1, 1, :] = 9
    S[1, 1, w - 1] = 0
    m = lib.Matcher(W, H, census=5, ndisp=w, npaths=8)
    d_lo = np.arange(H, dtype=np.int32) * 3
    dint, dsub = m.wta(_dev(S.astype(np.int16)), d_lo=_dev(d_lo))
    torch.cuda.synchronize()
    wi, ws = oracle.wta(S, d_lo)
    np.testing.assert_array_equal(_np_u16(dint), wi)
    np.testing.assert_array_equal(dsub.cpu().numpy(), ws)


def _road(name, seed):
    p = synth.make_pair(synth.scene_for_config(name, seed), seed)
    return p, synth.CONFIGS[name]


def _full_parity(lib, name, seed, d_lo=None):
    import torch
    p, c = _road(name, seed)
    H, W = p.left.shape
    m = lib.Matcher(W, H, census=c["census"], ndisp=c["ndisp"], npaths=c["npaths"],
                    p1=c["p1"], p2=c["p2"])
    dl = None if d_lo is None else _dev(d_lo)
    cost = m.cost(_dev(p.left), _dev(p.right), d_lo=dl)
    dint, dsub = m.aggregate_wta(cost, d_lo=dl)
    mi, ms = m.match(_dev(p.left), _dev(p.right), d_lo=dl)
    # the split calls bench.py times
    paths = m.aggregate_paths(cost)
    bi, bs = m.wta_paths(paths, d_lo=dl)
    torch.cuda.synchronize()
    n, w = c["census"], c["ndisp"]
    want_c = oracle.cost(oracle.census(p.left, n), oracle.census(p.right, n), n, w, d_lo)
    np.testing.assert_array_equal(cost.cpu().numpy(), want_c)
    want_S = oracle.sum_paths(want_c, c["npaths"], c["p1"], c["p2"])
    wi, ws = oracle.wta(want_S, d_lo)
    for a, b in ((dint, dsub), (mi, ms), (bi, bs)):
        np.testing.assert_array_equal(_np_u16(a), wi)
        assert np.abs(b.cpu().numpy() - ws).max() <= SUB_TOL
        np.testing.assert_array_equal(b.cpu().numpy(), ws)
    return m, cost, want_S


def test_road320_census5_4paths_full(lib):
    """320x240, census 5x5, 4 paths, disparities 0..31: every output."""
    m, cost, want_S = _full_parity(lib, "road320", 1000)
    import torch
    S = m.aggregate(cost)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(_np_u16(S).astype(np.uint32), want_S)


def test_road1280_census7_8paths_full(lib):
    """1280x720, census 7x7, 8 paths, disparities 0..127 (the benchmarked
    workload and launch configuration): every output."""
    _full_parity(lib, "road1280", 2000)


def test_road1920_census7_8paths_full(lib):
    """1920x1080, census 7x7, 8 paths, disparities 0..191 (twelve values per
    lane, the widest frame of the batched and learned-window workloads):
    every output of the plain full-range path."""
    _full_parity(lib, "road1920", 2001)


def test_road1280_row_windows_full(lib):
    """1280x720 with per-row windows of width 24 centred on the road model."""
    p, c = _road("road1280_pt", 3000)
    a0, a1, phi = p.road_params
    d_lo = oracle.window_from_road(a0, a1, phi, 1280, 720, 24, mode=0)
    _full_parity(lib, "road1280_pt", 3000, d_lo=d_lo)


def test_window_helper_matches_oracle(lib):
    for a0, a1, phi, w, mode, delta in [(7.8, 0.0996, 0.03, 24, 0, 0.0),
                                        (7.8, 0.0996, 0.05, 24, 1, 3.0),
                                        (2.6, 0.0996, -0.02, 32, 1, 1.5)]:
        got = lib.sgm_window_from_road(a0, a1, phi, 1280, 720, w, mode, delta).numpy()
        want = oracle.window_from_road(a0, a1, phi, 1280, 720, w, mode, delta)
        np.testing.assert_array_equal(got, want)


def test_repeatable_bitwise(lib):
    import torch
    p, c = _road("road320", 1001)
    m = lib.Matcher(320, 240, census=5, ndisp=32, npaths=4)
    outs = []
    for _ in range(3):
        a, b = m.match(_dev(p.left), _dev(p.right))
        torch.cuda.synchronize()
        outs.append((a.cpu().numpy().copy(), b.cpu().numpy().copy()))
    for a, b in outs[1:]:
        np.testing.assert_array_equal(a, outs[0][0])
        np.testing.assert_array_equal(b, outs[0][1])


@pytest.mark.parametrize("shape", [(133, 41, 7, 128, 8), (70, 23, 7, 24, 8), (61, 27, 7, 48, 8)],
                         ids=lambda s: "x".join(map(str, s)))
def test_split_aggregate_paths_and_selection(lib, shape):
    """sgm_aggregate_paths (all directions, one launch) + sgm_wta_paths."""
    import torch
    W, H, n, w, R = shape
    p2 = 120 if w != 48 else 220  # 48: Cmax + P2 > 255 -> uint16 volumes
    L, Rimg = _rand_pair(W, H, 17 + w)
    d_lo = np.random.default_rng(w).integers(0, 4, size=H).astype(np.int32)
    m = lib.Matcher(W, H, census=n, ndisp=w, npaths=R, p1=10, p2=p2)
    cost = m.cost(_dev(L), _dev(Rimg), d_lo=_dev(d_lo))
    paths = m.aggregate_paths(cost)
    dint, dsub = m.wta_paths(paths, d_lo=_dev(d_lo))
    torch.cuda.synchronize()
    c = cost.cpu().numpy()
    esz = m.path_volumes()[0]
    assert esz == (1 if 48 + p2 <= 255 else 2)
    for r in range(R):
        got = m.path_volume(paths, r).cpu().numpy()
        got = got.view(np.uint16) if esz == 2 else got
        np.testing.assert_array_equal(got, oracle.path(c, r, 10, p2), err_msg="path %d" % r)
    wi, ws = oracle.wta(oracle.sum_paths(c, R, 10, p2), d_lo)
    np.testing.assert_array_equal(_np_u16(dint), wi)
    np.testing.assert_array_equal(dsub.cpu().numpy(), ws)


@pytest.mark.parametrize("lanes", [4, 8, 16])
@pytest.mark.parametrize("w", [16, 24, 32, 40, 48, 64])
def test_lane_mappings_match_oracle(lib, w, lanes):
    """Every lane mapping of the volume kernels (a scanline / a pixel carried
    by 4, 8 or 16 lanes; idle lanes where the window does not fill the
    group) on a ragged frame with row windows: each direction's L_r, the
    selection on the per-direction volumes, the fused and the whole-path
    calls; uint8 volumes, and uint16 ones (P2 = 220) at two widths."""
    import torch
    W, H, n = 77, 29, 7
    p2 = 220 if w in (24, 48) else 120
    L, Rimg = _rand_pair(W, H, 31 * w + lanes)
    d_lo = np.random.default_rng(w + lanes).integers(0, 5, size=H).astype(np.int32)
    m = lib.Matcher(W, H, census=n, ndisp=w, npaths=8, p1=10, p2=p2, lanes=lanes)
    want_lanes = lanes if (lanes == 16 or any(lanes * v >= w and w % v == 0
                                              for v in ((4, 8) if lanes == 8 else (4, 8, 12, 16)))) else 16
    assert m.lanes == want_lanes
    dl = _dev(d_lo)
    cost = m.cost(_dev(L), _dev(Rimg), d_lo=dl)
    paths = m.aggregate_paths(cost)
    bi, bs = m.wta_paths(paths, d_lo=dl)
    fi, fs = m.aggregate_wta(cost, d_lo=dl)
    mi, ms = m.match(_dev(L), _dev(Rimg), d_lo=dl)
    torch.cuda.synchronize()
    c = cost.cpu().numpy()
    np.testing.assert_array_equal(c, oracle.cost(oracle.census(L, n), oracle.census(Rimg, n), n, w, d_lo))
    esz = m.path_volumes()[0]
    for r in range(8):
        got = m.path_volume(paths, r).cpu().numpy()
        got = got.view(np.uint16) if esz == 2 else got
        np.testing.assert_array_equal(got, oracle.path(c, r, 10, p2), err_msg="path %d" % r)
    wi, ws = oracle.wta(oracle.sum_paths(c, 8, 10, p2), d_lo)
    for a, b in ((bi, bs), (fi, fs), (mi, ms)):
        np.testing.assert_array_equal(_np_u16(a), wi)
        assert np.abs(b.cpu().numpy() - ws).max() <= SUB_TOL
        np.testing.assert_array_equal(b.cpu().numpy(), ws)


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_slot_orders_match_oracle(lib, lanes):
    """Both dispatch orders of the aggregation's direction slots, with each
    lane count, on a ragged row-window frame: every direction's L_r and the
    disparities equal the oracle's."""
    import torch
    W, H, n, w = 93, 41, 7, 24
    L, Rimg = _rand_pair(W, H, 577 + lanes)
    d_lo = np.random.default_rng(lanes).integers(0, 7, size=H).astype(np.int32)
    c = oracle.cost(oracle.census(L, n), oracle.census(Rimg, n), n, w, d_lo)
    wi, ws = oracle.wta(oracle.sum_paths(c, 8, 10, 120), d_lo)
    dl = _dev(d_lo)
    for order in (0, 1):
        m = lib.Matcher(W, H, census=n, ndisp=w, npaths=8, p1=10, p2=120, lanes=lanes, order=order)
        assert (m.lanes, m.order) == (lanes, order)
        cost = m.cost(_dev(L), _dev(Rimg), d_lo=dl)
        paths = m.aggregate_paths(cost)
        mi, ms = m.match(_dev(L), _dev(Rimg), d_lo=dl)
        torch.cuda.synchronize()
        for r in range(8):
            np.testing.assert_array_equal(m.path_volume(paths, r).cpu().numpy(), oracle.path(c, r, 10, 120),
                                          err_msg="order %d path %d" % (order, r))
        np.testing.assert_array_equal(_np_u16(mi), wi)
        np.testing.assert_array_equal(ms.cpu().numpy(), ws)


def test_single_pair_autotune_keeps_results(lib, tmp_path):
    """sgm_autotune times the lane mappings, caches the choice, and the
    tuned plan gives the oracle's disparities."""
    import torch
    p, c = _road("road1280_pt", 3001)
    H, W = p.left.shape
    a0, a1, phi = p.road_params
    d_lo = oracle.window_from_road(a0, a1, phi, W, H, 24, mode=0)
    m = lib.Matcher(W, H, census=7, ndisp=24, npaths=8)
    cache = tmp_path / "tune.txt"
    L, Rt, dl = _dev(p.left), _dev(p.right), _dev(d_lo)
    lanes = m.autotune(L, Rt, d_lo=dl, cache_path=cache)
    assert lanes in (4, 8, 16) and m.lanes == lanes and m.order in (0, 1)
    assert len(cache.read_text().splitlines()) == 1
    m2 = lib.Matcher(W, H, census=7, ndisp=24, npaths=8)
    assert m2.autotune(L, Rt, d_lo=dl, cache_path=cache) == lanes  # read back
    assert m2.order == m.order
    assert len(cache.read_text().splitlines()) == 1
    dint, dsub = m.match(L, Rt, d_lo=dl)
    torch.cuda.synchronize()
    n = 7
    want_c = oracle.cost(oracle.census(p.left, n), oracle.census(p.right, n), n, 24, d_lo)
    wi, ws = oracle.wta(oracle.sum_paths(want_c, 8, 10, 120), d_lo)
    np.testing.assert_array_equal(_np_u16(dint), wi)
    np.testing.assert_array_equal(dsub.cpu().numpy(), ws)


def test_single_pair_step_replays_in_a_graph(lib):
    """The split single-pair step (sgm_cost, sgm_aggregate_paths,
    sgm_wta_paths, as the benchmark times it) captured once in a HIP graph:
    every replay on new images copied into the captured buffers, with eager
    work and synchronisations in between, equals the oracle and the eager
    step bit for bit."""
    import torch
    W, H, D = 150, 70, 48
    m = lib.Matcher(W, H, census=7, ndisp=D, npaths=8, p1=10, p2=120)
    left = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    right = torch.empty_like(left)
    cost = m.new_volume(torch.uint8)
    paths = m.new_paths()
    dint = torch.empty((H, W), dtype=torch.int16, device="cuda")
    dsub = torch.empty((H, W), dtype=torch.float32, device="cuda")

    def step():
        m.cost(left, right, cost=cost)
        m.aggregate_paths(cost, paths)
        m.wta_paths(paths, disp_int=dint, disp_sub=dsub)

    L0, R0 = _rand_pair(W, H, 5)
    left.copy_(torch.from_numpy(L0))
    right.copy_(torch.from_numpy(R0))
    step()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for seed in (11, 12, 13):
        L, R = _rand_pair(W, H, seed)
        left.copy_(torch.from_numpy(L))
        right.copy_(torch.from_numpy(R))
        dint.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        gi, gs = dint.clone(), dsub.clone()
        step()  # eager, same buffers
        torch.cuda.synchronize()
        assert torch.equal(gi, dint) and torch.equal(gs, dsub), seed
        wi, ws = oracle.sgm(L, R, 7, D, 8, 10, 120)
        np.testing.assert_array_equal(_np_u16(gi), wi)
        np.testing.assert_array_equal(gs.cpu().numpy(), ws)


def test_injected_launch_fault_then_recovery(lib):
    """An armed launch fault fails exactly one call (nothing enqueued); the
    next call runs normally and matches the oracle."""
    import torch
    L, R = _rand_pair(40, 12, 99)
    m = lib.Matcher(40, 12, census=5, ndisp=16, npaths=4, p1=10, p2=120)
    Ld, Rd = torch.from_numpy(L).cuda(), torch.from_numpy(R).cuda()
    assert lib.library().sgm_debug_inject_fault(1) == 0
    with pytest.raises(lib.SgmError):
        m.match(Ld, Rd)
    di, ds = m.match(Ld, Rd)
    torch.cuda.synchronize()
    wi, _ = oracle.sgm(L, R, 5, 16, 4, 10, 120)
    np.testing.assert_array_equal(di.cpu().numpy().view(np.uint16), wi)
