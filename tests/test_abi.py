"""Host-only checks of the C ABI: the library loads, exports every function
that include/sgm.h declares, and rejects bad arguments before enqueueing
anything (none of these calls needs a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def sgm():
    from paper_2012_10802_amd import sgm as mod
    return mod


def test_every_declared_symbol_is_exported(sgm):
    names = _declared("sgm.h")
    assert "sgm_plan" in names and "sgm_match" in names
    lib = ctypes.CDLL(sgm.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _params(**kw):
    from paper_2012_10802_amd.sgm import sgm_params
    d = dict(width=64, height=32, census=7, ndisp=64, npaths=8, p1=10, p2=120, flags=0)
    d.update(kw)
    return sgm_params(**d)


def _plan_status(sgm, **kw):
    h = ctypes.c_void_p()
    st = sgm.library().sgm_plan(ctypes.byref(_params(**kw)), ctypes.byref(h))
    if st == 0:
        sgm.library().sgm_plan_free(h)
    return st


@pytest.mark.parametrize("kw,want", [
    ({}, 0),
    ({"width": 0}, -1),
    ({"height": -3}, -1),
    ({"census": 9}, -2),
    ({"census": 4}, -2),
    ({"ndisp": 0}, -1),
    ({"ndisp": 257}, -1),
    ({"npaths": 6}, -2),
    ({"p1": 11, "p2": 10}, -1),
    ({"p1": -1}, -1),
    ({"p2": 8200}, -1),
    ({"p2": 5430}, -1),
    ({"p1": 5, "p2": 5397}, 0),
    ({"flags": 1}, -1),
    ({"width": 40000, "height": 40000, "ndisp": 8}, -2),
    ({"census": 3, "ndisp": 256, "npaths": 4, "p2": 4000}, 0),
    ({"census": 7, "npaths": 8, "p2": 5429}, -1),
    ({"census": 7, "npaths": 8, "p2": 5428}, 0),
])
def test_plan_validation(sgm, kw, want):
    assert _plan_status(sgm, **kw) == want


@pytest.mark.parametrize("kw,want", [
    # uint8 volumes (Cmax + P2 = 168): any W*H*ndisp below 2^31
    ({"width": 4096, "height": 2304, "ndisp": 128}, 0),
    # uint16 volumes (Cmax + P2 = 268): 4096x2304x128 = 1.2e9 values is more
    # than 2^30, so a dropped store (byte 2^31) would land inside the volume
    ({"width": 4096, "height": 2304, "ndisp": 128, "p2": 220}, -2),
    ({"width": 4096, "height": 2048, "ndisp": 128, "p2": 220}, -2),   # exactly 2^30
    ({"width": 4096, "height": 2047, "ndisp": 128, "p2": 220}, 0),    # 2^30 - 4096*128
])
def test_plan_rejects_uint16_volumes_reaching_the_drop_offset(sgm, kw, want):
    assert _plan_status(sgm, **kw) == want
    if want:
        assert b"2^30" in sgm.library().sgm_last_error()


def test_aggregate_path_rejects_volumes_reaching_the_drop_offset(sgm):
    """sgm_aggregate_path always writes uint16: a plan with 2^30 or more
    values is refused there before anything is enqueued."""
    lib = sgm.library()
    dummy = ctypes.c_void_p(256)
    plan = sgm.sgm_plan(4096, 2304, 7, 128, 8, 10, 120)
    try:
        assert lib.sgm_aggregate_path(plan, dummy, 0, dummy, None) == -2
        assert b"2^30" in lib.sgm_last_error()
    finally:
        sgm.sgm_plan_free(plan)


def test_batch_plan_rejects_uint16_volumes_reaching_the_drop_offset(sgm):
    lib = sgm.library()

    def status(W, H, w, p2):
        prm = sgm.sgm_batch_params(7, 8, 10, p2, 0)
        arr = (sgm.sgm_pair * 1)(sgm.sgm_pair(W, H, w, W, 256, 256, None, 256, None))
        h = ctypes.c_void_p()
        st = lib.sgm_batch_plan(ctypes.byref(prm), arr, 1, ctypes.byref(h))
        if st == 0:
            lib.sgm_batch_free(h)
        return st

    assert status(4096, 2304, 128, 220) == -2
    # accepted by validation; without a GPU the plan's pinned queue cannot
    # be allocated afterwards (SGM_ERR_HIP)
    assert status(4096, 2047, 128, 220) in (0, -3)
    assert status(4096, 2304, 128, 120) in (0, -3)


@pytest.mark.parametrize("lanes,order,want_status,want", [
    (0, 0, 0, (16, 0)),
    (8, 1, 0, (8, 1)),
    (4, 1, 0, (4, 1)),
    (4, 0, 0, (4, 0)),
    (8, 2, -1, None),
    (8, -1, -1, None),
    (5, 0, -1, None),
])
def test_plan_tuning_round_trip(sgm, lanes, order, want_status, want):
    """sgm_plan_tuned keeps the lane count (w = 64 serves 4, 8 and 16) and
    the slot order, rejects orders outside {0, 1} and unknown lane counts,
    and sgm_plan_get_tuning reports both."""
    lib = sgm.library()
    h = ctypes.c_void_p()
    t = sgm.sgm_tuning(0, order, lanes)
    st = lib.sgm_plan_tuned(ctypes.byref(_params()), ctypes.byref(t), ctypes.byref(h))
    assert st == want_status
    if st != 0:
        return
    try:
        got = sgm.sgm_tuning()
        assert lib.sgm_plan_get_tuning(h, ctypes.byref(got)) == 0
        assert (got.lanes, got.order, got.waves_per_cu) == (want[0], want[1], 0)
    finally:
        lib.sgm_plan_free(h)


def test_error_strings(sgm):
    lib = sgm.library()
    assert lib.sgm_status_str(-4) == b"SGM_ERR_WORKSPACE"
    assert _plan_status(sgm, npaths=5) == -2
    assert b"npaths" in lib.sgm_last_error()


def test_workspace_size_and_checks(sgm):
    lib = sgm.library()
    plan = sgm.sgm_plan(1280, 720, 7, 128, 8, 10, 120)
    try:
        n = sgm.sgm_workspace_size(plan)
        # census codes + cost + 8 uint8 per-path volumes
        assert n >= 2 * 1280 * 720 * 8 + 9 * 1280 * 720 * 128
        dummy = ctypes.c_void_p(256)
        # null inputs and a short workspace are refused before any launch
        assert lib.sgm_cost(plan, None, dummy, 1280, None, dummy, dummy, n, None) == -1
        assert lib.sgm_cost(plan, dummy, dummy, 1000, None, dummy, dummy, n, None) == -1
        assert lib.sgm_aggregate(plan, dummy, dummy, dummy, n - 1, None) == -4
        assert lib.sgm_aggregate(plan, dummy, dummy, ctypes.c_void_p(258), n, None) == -1
        assert lib.sgm_aggregate_path(plan, dummy, 8, dummy, None) == -1
        assert lib.sgm_wta(plan, None, None, dummy, None, None) == -1
        assert lib.sgm_match(plan, dummy, dummy, 1280, None, None, None, dummy, n, None) == -1
        assert lib.sgm_aggregate(None, dummy, dummy, dummy, n, None) == -1
    finally:
        sgm.sgm_plan_free(plan)


def test_noalloc_match_rejects_plans_beyond_its_scratch(sgm):
    """sgm_match_noalloc refuses, before any HIP call, plans whose workspace
    exceeds the library's scratch array, and null arguments."""
    lib = sgm.library()
    limit = 64 << 20
    dummy = ctypes.c_void_p(256)
    small = sgm.sgm_plan(320, 240, 5, 32, 4, 10, 120)
    big = sgm.sgm_plan(1280, 720, 7, 128, 8, 10, 120)
    try:
        assert sgm.sgm_workspace_size(small) <= limit < sgm.sgm_workspace_size(big)
        assert lib.sgm_match_noalloc(big, dummy, dummy, 1280, None, dummy, None, None) == -4
        assert b"scratch" in lib.sgm_last_error()
        assert lib.sgm_match_noalloc(None, dummy, dummy, 320, None, dummy, None, None) == -1
        assert lib.sgm_match_noalloc(small, None, dummy, 320, None, dummy, None, None) == -1
        assert lib.sgm_match_noalloc(small, dummy, dummy, 320, None, None, None, None) == -1
    finally:
        sgm.sgm_plan_free(small)
        sgm.sgm_plan_free(big)


def test_window_helper_host(sgm):
    import math
    import oracle
    d = sgm.sgm_window_from_road(20.0, 0.1, 0.0, 640, 480, 24, 0).numpy()
    cy = 239.5
    assert list(d) == [max(0, math.floor(20.0 + 0.1 * (v - cy) + 0.5) - 12) for v in range(480)]
    for args in [(7.8, 0.0996, 0.05, 1280, 720, 24, 1, 3.0), (2.6, 0.09, -0.03, 640, 480, 32, 1, 0.5),
                 (44.0, 0.15, 0.02, 1920, 1080, 16, 0, 0.0)]:
        np.testing.assert_array_equal(sgm.sgm_window_from_road(*args).numpy(),
                                      oracle.window_from_road(*args))
    lib = sgm.library()
    assert lib.sgm_window_from_road(1.0, 1.0, 0.0, 10, 10, 4, 2, 0.0, None) == -1
    with pytest.raises(sgm.SgmError):
        sgm.sgm_window_from_road(float("nan"), 1.0, 0.0, 10, 10, 4, 0)


def test_batch_plan_validation(sgm):
    lib = sgm.library()
    prm = sgm.sgm_batch_params(7, 8, 10, 120, 0)

    def status(*pairs, prm=prm):
        arr = (sgm.sgm_pair * len(pairs))(*pairs)
        h = ctypes.c_void_p()
        st = lib.sgm_batch_plan(ctypes.byref(prm), arr, len(pairs), ctypes.byref(h))
        if st == 0:
            lib.sgm_batch_free(h)
        return st

    ok = sgm.sgm_pair(64, 32, 64, 64, 256, 256, None, 256, None)
    assert status(sgm.sgm_pair(64, 32, 100, 64, 256, 256, None, 256, None)) == -2  # 100 % 8
    assert status(sgm.sgm_pair(64, 32, 64, 60, 256, 256, None, 256, None)) == -1  # pitch
    assert status(sgm.sgm_pair(64, 32, 64, 64, None, 256, None, 256, None)) == -1  # NULL
    assert status(ok, sgm.sgm_pair(0, 32, 64, 64, 256, 256, None, 256, None)) == -1
    assert status(ok, prm=sgm.sgm_batch_params(9, 8, 10, 120, 0)) == -2
    assert status(ok, prm=sgm.sgm_batch_params(7, 8, 130, 120, 0)) == -1
    h = ctypes.c_void_p()
    arr = (sgm.sgm_pair * 1)(ok)
    assert lib.sgm_batch_plan(ctypes.byref(prm), arr, 0, ctypes.byref(h)) == -1
    assert lib.sgm_batch_run(None, None, 0, None) == -1
    assert lib.sgm_batch_launch(None, None) == -1


def test_fallback_rects_host_logic_matches_oracle():
    """The product's rectangle selection (host code, numpy, from per-row
    statistics) against the oracle's plain loops over the mask."""
    from oracle import cnn as ocnn
    from paper_2012_10802_amd import learned_window as lw
    rng = np.random.default_rng(17)
    for trial in range(300):
        H, W = int(rng.integers(1, 90)), int(rng.integers(1, 400))
        dens = [0.0, 0.0005, 0.005, 0.05, 0.5][trial % 5]
        mask = (rng.random((H, W)) < dens).astype(np.uint8)
        if trial % 7 == 0:
            mask[:, :int(rng.integers(0, W + 1))] = 0  # fallback only on the right
        stats = np.zeros((3, H), np.int64)
        stats[0] = mask.sum(axis=1)
        cols = np.arange(W)
        stats[1] = np.where(mask > 0, cols, W).min(axis=1)
        stats[2] = np.where(mask > 0, cols, -1).max(axis=1)
        margin, D = int(rng.integers(0, 20)), int(rng.choice([16, 64, 192]))
        frac = float(rng.choice([0.2, 0.5, 1.0]))
        assert lw.fallback_rects(stats, W, D, 3, margin, frac) == ocnn.fallback_rects(mask, margin, frac, D, 3)


def test_window_batch_needs_width_16():
    """sgm_match_win_batch refuses plans other than 16 disparities before it
    touches any buffer (SGM_ERR_UNSUPPORTED)."""
    import ctypes
    from paper_2012_10802_amd import sgm
    lib = sgm.library()
    plan = sgm.sgm_plan(64, 32, 7, 12, 8, 10, 120)
    try:
        rc = lib.sgm_match_win_batch(plan, None, None, 64, 64 * 32, None, 2, None, None, None, 0, None)
        assert rc == -2
        b = ctypes.c_size_t()
        assert lib.sgm_workspace_size_win_batch(plan, 3, ctypes.byref(b)) == 0
        # each pair's slice: the plan's workspace, then its window starts as bytes
        assert b.value == 3 * (sgm.sgm_workspace_size(plan) + (64 * 32 + 255) // 256 * 256)
        assert lib.sgm_workspace_size_win_batch(plan, 0, ctypes.byref(b)) == -1
    finally:
        sgm.sgm_plan_free(plan)


def test_cnn_and_window_calls_validate_before_launch():
    """Size, threshold and rectangle checks of the network / window-map /
    fallback calls return their status before anything is enqueued (dummy
    non-NULL pointers are never touched)."""
    import ctypes
    from paper_2012_10802_amd import sgm
    lib = sgm.library()
    d = ctypes.c_void_p(256)  # never dereferenced: every call below fails validation
    f = ctypes.c_float
    # sizes
    assert lib.sgm_cnn_forward(d, d, d, 0, 8, 1, d, d, None) == -1
    assert lib.sgm_cnn_forward(d, d, d, 1 << 16, 1 << 12, 1, d, d, None) == -2
    assert lib.sgm_cnn_infer(d, d, d, 0, 8, 1, d, None) == -1
    assert lib.sgm_cnn_infer(d, d, d, 8, 8, 1 << 16, d, None) == -2
    assert lib.sgm_cnn_infer(d, d, ctypes.c_void_p(258), 8, 8, 1, d, None) == -1  # x0 misaligned
    assert lib.sgm_cnn_prepare_input(d, d, 8, 8, 0, d, None) == -1
    assert lib.sgm_cnn_loss(d, d, d, 8, -1, 1, d, None, None) == -1
    assert lib.sgm_cnn_backward(d, d, d, d, 8, 8, 1, d, d, 0, None) == -4  # scratch too small
    assert lib.sgm_cnn_adam(d, d, d, d, 0, f(1e-3), f(0.9), f(0.999), f(1e-8), d, d, None) == -1
    # window map: NaN threshold, window wider than the range
    assert lib.sgm_window_map(d, d, 4, 4, 16, 16, 192, 16, f(float("nan")), 0, d, None, None, None, None) == -1
    assert lib.sgm_window_map(d, d, 4, 4, 16, 16, 8, 16, f(0.5), 0, d, None, None, None, None) == -1
    # fallback merge: rectangle outside the frame, too many rows
    assert lib.sgm_fallback_merge(d, d, None, 100, 50, 40, 20, 0, 10, d, None, None) == -1
    assert lib.sgm_fallback_merge(d, d, None, 100, 50, 0, 10, 95, 10, d, None, None) == -1
    assert lib.sgm_fallback_merge(d, d, None, 4, 70000, 0, 70000, 0, 4, d, None, None) == -2
    assert lib.sgm_label_downsample4(d, 3, 8, d, None) == -1


def test_injected_faults_fail_before_anything_is_enqueued():
    """The failure-handling hook: an armed launch fault makes the next
    launching call return SGM_ERR_HIP with nothing enqueued (the dummy
    buffers below are never touched), an armed allocation fault makes the
    next batch plan fail; kinds outside 0..2 are rejected."""
    import ctypes
    from paper_2012_10802_amd import sgm
    lib = sgm.library()
    assert lib.sgm_debug_inject_fault(3) == -1
    plan = sgm.sgm_plan(64, 32, 7, 16, 8, 10, 120)
    try:
        ws = sgm.sgm_workspace_size(plan)
        d = ctypes.c_void_p(1 << 20)
        assert lib.sgm_debug_inject_fault(1) == 0
        rc = lib.sgm_cost(plan, d, d, 64, None, d, d, ws, None)
        assert rc == -3 and b"injected" in lib.sgm_last_error()
    finally:
        sgm.sgm_plan_free(plan)
    assert lib.sgm_debug_inject_fault(2) == 0
    pairs = (sgm.sgm_pair * 1)()
    pairs[0] = sgm.sgm_pair(64, 32, 16, 64, 1 << 20, 1 << 20, None, 1 << 20, None)
    prm = sgm.sgm_batch_params(7, 8, 10, 120, 0)
    h = ctypes.c_void_p()
    rc = lib.sgm_batch_plan(ctypes.byref(prm), pairs, 1, ctypes.byref(h))
    assert rc == -3 and b"injected" in lib.sgm_last_error()
    assert lib.sgm_debug_inject_fault(0) == 0


def test_road_calls_validate_before_launch():
    """The road-model calls (fit, windows, transformation) check sizes,
    bounds, alignment and workspace before anything is enqueued (dummy
    non-NULL pointers are never touched); the fit record is 64 bytes."""
    import ctypes
    from paper_2012_10802_amd import sgm
    lib = sgm.library()
    d = ctypes.c_void_p(1 << 20)
    f = ctypes.c_float
    n = ctypes.c_size_t()
    assert lib.sgm_road_workspace_size(1920, 1080, 16, ctypes.byref(n)) == 0 and n.value > 0
    assert lib.sgm_road_workspace_size(0, 1080, 16, ctypes.byref(n)) == -1
    assert lib.sgm_road_workspace_size(8, 8, 70000, ctypes.byref(n)) == -2
    assert lib.sgm_road_workspace_size(1 << 16, 1 << 15, 1, ctypes.byref(n)) == -2
    ws = sgm.road_workspace_size(64, 48, 2)
    ninf = float("-inf")
    assert lib.sgm_road_fit_batch(None, None, 64, 48, 2, f(0.0), ninf, None, float("inf"), d, d, ws, None) == -1
    assert lib.sgm_road_fit_batch(d, None, 64, 48, 2, f(float("nan")), ninf, None, float("inf"), d, d, ws, None) == -1
    assert lib.sgm_road_fit_batch(d, None, 64, 48, 2, f(0.0), float("nan"), None, float("inf"), d, d, ws, None) == -1
    assert lib.sgm_road_fit_batch(d, None, 64, 48, 2, f(0.0), ninf, None, float("inf"), d, None, ws, None) == -1
    assert lib.sgm_road_fit_batch(d, None, 64, 48, 2, f(0.0), ninf, None, float("inf"), d, ctypes.c_void_p((1 << 20) + 16), ws,
                                  None) == -1
    assert lib.sgm_road_fit_batch(d, None, 64, 48, 2, f(0.0), ninf, None, float("inf"), d, d, ws - 1, None) == -4
    assert lib.sgm_road_fit_batch(ctypes.c_void_p((1 << 20) + 2), None, 64, 48, 2, f(0.0), ninf, None, float("inf"), d, d, ws,
                                  None) == -1
    assert lib.sgm_road_fit_batch(d, None, 64, 48, 2, f(0.0), ninf, d, -1.0, d, d, ws, None) == -1
    assert lib.sgm_road_fit_batch(d, None, 64, 48, 2, f(0.0), ninf, d, float("nan"), d, d, ws, None) == -1
    assert lib.sgm_road_fit_batch(d, None, 64, 48, 2, f(0.0), ninf, ctypes.c_void_p((1 << 20) + 4), 1.0, d, d, ws,
                                  None) == -1
    assert lib.sgm_road_window_batch(d, 64, 48, 2, 0, 0, 0.0, 1.0, d, None) == -1
    assert lib.sgm_road_window_batch(d, 64, 48, 2, 24, 2, 0.0, 1.0, d, None) == -1
    assert lib.sgm_road_window_batch(d, 64, 48, 2, 24, 1, float("inf"), 1.0, d, None) == -1
    assert lib.sgm_road_window_batch(d, 64, 48, 2, 24, 1, 0.0, 0.0, d, None) == -1
    assert lib.sgm_road_window_batch(d, 64, 48, 2, 24, 1, 0.0, float("nan"), d, None) == -1
    assert lib.sgm_road_window_batch(None, 64, 48, 2, 24, 1, 0.0, 1.0, d, None) == -1
    assert lib.sgm_disparity_transform_batch(d, d, 64, 48, 2, float("nan"), d, None) == -1
    assert lib.sgm_disparity_transform_batch(d, d, 64, -48, 2, 0.0, d, None) == -1
    assert lib.sgm_disparity_transform_batch(d, d, 64, 48, 2, 0.0, None, None) == -1
    assert lib.sgm_road_window_map_batch(d, 64, 48, 2, 0, 1.0, d, None) == -1
    assert lib.sgm_road_window_map_batch(d, 64, 48, 2, 16, -1.0, d, None) == -1
    assert lib.sgm_road_window_map_batch(None, 64, 48, 2, 16, 1.0, d, None) == -1
    assert lib.sgm_road_mask_batch(d, d, 64, 48, 2, float("nan"), 0.0, d, None) == -1
    assert lib.sgm_road_mask_batch(d, None, 64, 48, 2, 1.0, 0.0, d, None) == -1
    assert lib.sgm_road_mask_batch(d, d, 64, 48, 0, 1.0, 0.0, d, None) == -1
    E = lib.sgm_road_energy_batch
    inf = float("inf")
    assert E(d, None, 64, 48, 2, f(0.0), ninf, None, inf, None, 5, d, d, ws, None) == -1  # phi NULL
    assert E(d, None, 64, 48, 2, f(0.0), ninf, None, inf, d, 5, None, d, ws, None) == -1  # energy NULL
    assert E(d, None, 64, 48, 2, f(0.0), ninf, None, inf, d, 0, d, d, ws, None) == -1
    assert E(d, None, 64, 48, 2, f(0.0), ninf, None, inf, d, 65537, d, d, ws, None) == -1
    assert E(d, None, 64, 48, 2, f(float("nan")), ninf, None, inf, d, 5, d, d, ws, None) == -1
    assert E(d, None, 64, 48, 2, f(0.0), ninf, d, -1.0, d, 5, d, d, ws, None) == -1
    assert E(d, None, 64, 48, 2, f(0.0), ninf, None, inf, ctypes.c_void_p((1 << 20) + 4), 5, d, d, ws, None) == -1
    assert E(d, None, 64, 48, 2, f(0.0), ninf, None, inf, d, 5, ctypes.c_void_p((1 << 20) + 4), d, ws, None) == -1
    assert E(d, None, 64, 48, 2, f(0.0), ninf, None, inf, d, 5, d, d, ws - 1, None) == -4
    assert E(d, None, 64, 48, 0, f(0.0), ninf, None, inf, d, 5, d, d, ws, None) == -1
    # an armed launch fault fails the fit and the curve with nothing enqueued
    assert lib.sgm_debug_inject_fault(1) == 0
    assert lib.sgm_road_fit_batch(d, None, 64, 48, 2, f(0.0), ninf, None, float("inf"), d, d, ws, None) == -3
    assert lib.sgm_debug_inject_fault(1) == 0
    assert E(d, None, 64, 48, 2, f(0.0), ninf, None, inf, d, 5, d, d, ws, None) == -3
    assert lib.sgm_debug_inject_fault(0) == 0


def test_pothole_calls_validate_before_launch():
    """Threshold / labelling calls check bins, range, alignment and
    workspace before anything is enqueued (dummy pointers never touched)."""
    import ctypes
    from paper_2012_10802_amd import sgm
    lib = sgm.library()
    d = ctypes.c_void_p(1 << 20)
    n = ctypes.c_size_t()
    assert lib.sgm_pothole_workspace_size(128, 16, ctypes.byref(n)) == 0 and n.value == 16 * 2 * 128 * 4 * 8
    assert lib.sgm_pothole_workspace_size(1, 16, ctypes.byref(n)) == -1
    assert lib.sgm_pothole_workspace_size(513, 16, ctypes.byref(n)) == -1
    ws = sgm.pothole_workspace_size(64, 2)
    T = lib.sgm_pothole_threshold_batch
    assert T(None, None, 64, 48, 2, 0.0, 16.0, 64, 2.36, d, None, d, ws, None) == -1
    assert T(d, None, 64, 48, 2, 16.0, 16.0, 64, 2.36, d, None, d, ws, None) == -1
    assert T(d, None, 64, 48, 2, 0.0, float("inf"), 64, 2.36, d, None, d, ws, None) == -1
    assert T(d, None, 64, 48, 2, 0.0, 16.0, 1, 2.36, d, None, d, ws, None) == -1
    assert T(d, None, 64, 48, 2, 0.0, 16.0, 64, float("nan"), d, None, d, ws, None) == -1
    assert T(d, None, 64, 48, 2, 0.0, 16.0, 64, 2.36, d, None, d, ws - 8, None) == -4
    assert T(d, None, 64, 48, 2, 0.0, 16.0, 64, 2.36, d, None, ctypes.c_void_p((1 << 20) + 64), ws, None) == -1
    assert T(d, None, 64, 48, 2, 0.0, 16.0, 64, 2.36, d, ctypes.c_void_p((1 << 20) + 4), d, ws, None) == -1
    assert T(d, None, 0, 48, 2, 0.0, 16.0, 64, 2.36, d, None, d, ws, None) == -1
    L = lib.sgm_pothole_label_batch
    assert L(d, None, 64, 48, 2, None, d, None) == -1
    assert L(d, None, 64, 48, 2, d, ctypes.c_void_p((1 << 20) + 2), None) == -1
    assert L(d, None, 64, 48, 70000, d, d, None) == -2
    assert lib.sgm_debug_inject_fault(1) == 0
    assert L(d, None, 64, 48, 2, d, d, None) == -3
    assert lib.sgm_debug_inject_fault(0) == 0


def test_pothole_prune_validates_before_launch():
    import ctypes
    from paper_2012_10802_amd import sgm
    lib = sgm.library()
    d = ctypes.c_void_p(1 << 20)
    P = lib.sgm_pothole_prune_batch
    assert P(None, 64, 48, 2, d, None) == -1
    assert P(d, 64, 48, 2, None, None) == -1
    assert P(d, 0, 48, 2, d, None) == -1
    assert P(d, 64, 48, 70000, d, None) == -2
    assert P(ctypes.c_void_p((1 << 20) + 2), 64, 48, 2, d, None) == -1
    assert P(d, 64, 48, 2, ctypes.c_void_p((1 << 20) + 2), None) == -1
    assert lib.sgm_debug_inject_fault(1) == 0
    assert P(d, 64, 48, 2, d, None) == -3
    assert lib.sgm_debug_inject_fault(0) == 0


def test_slic_calls_validate_before_launch():
    import ctypes
    from paper_2012_10802_amd import sgm
    lib = sgm.library()
    d = ctypes.c_void_p(1 << 20)
    n = ctypes.c_size_t()
    assert lib.sgm_slic_workspace_size(1920, 1080, 16, 16, ctypes.byref(n)) == 0
    assert n.value == 120 * 68 * 16 * 4 * 8 + 16 * 100 * 8  # accumulators, then residuals of 100 rounds
    assert lib.sgm_slic_workspace_size(64, 48, 1, 1, ctypes.byref(n)) == -1
    assert lib.sgm_slic_workspace_size(64, 48, 257, 1, ctypes.byref(n)) == -1
    ws = sgm.slic_workspace_size(64, 48, 8, 2)
    B = lib.sgm_slic_batch
    assert B(d, None, 64, 48, 2, 8, 10.0, 5, 0.0, None, d, d, None, d, ws, None) == -1
    assert B(d, None, 64, 48, 2, 8, -1.0, 5, 0.0, None, d, d, d, d, ws, None) == -1
    assert B(d, None, 64, 48, 2, 8, float("nan"), 5, 0.0, None, d, d, d, d, ws, None) == -1
    assert B(d, None, 64, 48, 2, 8, 10.0, 0, 0.0, None, d, d, d, d, ws, None) == -1
    assert B(d, None, 64, 48, 2, 8, 10.0, 101, 0.0, None, d, d, d, d, ws, None) == -1
    for tol in (-0.5, float("nan"), float("inf")):
        assert B(d, None, 64, 48, 2, 8, 10.0, 5, tol, None, d, d, d, d, ws, None) == -1
    assert B(d, None, 64, 48, 2, 8, 10.0, 5, 0.0, ctypes.c_void_p((1 << 20) + 2), d, d, d, d, ws, None) == -1
    assert B(d, None, 64, 48, 2, 8, 10.0, 5, 0.0, None, d, d, d, d, ws - 8, None) == -4
    assert B(d, None, 64, 48, 2, 8, 10.0, 5, 0.0, None, d, d, ctypes.c_void_p((1 << 20) + 4), d, ws, None) == -1
    assert B(d, None, 64, 48, 2, 8, 10.0, 5, 0.0, None, d, d, d, None, ws, None) == -1
    assert B(d, None, 4, 300000, 1, 2, 10.0, 5, 0.0, None, d, d, d, d, ws, None) == -2
