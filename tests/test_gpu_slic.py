"""Parity of the superpixel step (SLIC of Sec. II-D, D3 of Sec. II-E) with
the CPU oracle, through the C ABI.

Every quantity is decided the same way on both sides: float64 distances
without fused multiply-add in the same order, integer sums for the means,
the same float64 divisions.  So labels, centres and D3 must match bit for
bit.
"""
import json
import os

import numpy as np
import pytest

from oracle import pothole as opd
from oracle import slic as oslic

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


def _same(got, D, S, m, iters, mask=None, tol=0.0, rounds=None):
    lab, d3, cen = (t.cpu().numpy() for t in got)
    info = {}
    wl, wd3, (cx, cy, cv) = oslic.slic(D, S, m, iters, mask, tol=tol, info=info)
    np.testing.assert_array_equal(lab, wl)
    np.testing.assert_array_equal(cen, np.stack([cx, cy, cv], 1))
    np.testing.assert_array_equal(d3, wd3)
    if rounds is not None:
        assert rounds == info["rounds"]


def test_hand_worked_maps(lib):
    with open(os.path.join(GOLD, "hand_slic.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        D = np.array(c["disp"], np.float32)
        lab, d3, cen = lib.slic(_dev(D), c["S"], c["m"], c["iters"])
        np.testing.assert_array_equal(lab.cpu().numpy()[0], c["labels"])
        np.testing.assert_array_equal(cen.cpu().numpy()[0], c["centres"])
        np.testing.assert_array_equal(d3.cpu().numpy()[0], c["d3"])


def _two_level(rng, H, W, holes=3):
    vv, uu = np.mgrid[0:H, 0:W]
    D = np.full((H, W), 10.0) + rng.normal(0, 0.4, (H, W))
    for _ in range(holes):
        cu, cv = rng.uniform(0, W), rng.uniform(0, H)
        ru, rv = rng.uniform(3, max(4, W / 5)), rng.uniform(2, max(3, H / 5))
        r2 = ((uu - cu) / ru) ** 2 + ((vv - cv) / rv) ** 2
        D = np.where(r2 < 1, D - 4 * (1 - r2), D)
    return D.astype(np.float32)


@pytest.mark.parametrize("H,W,S,m,iters", [(60, 90, 10, 5.0, 5), (37, 53, 8, 2.0, 10), (16, 16, 16, 1.0, 3),
                                           (45, 130, 17, 20.0, 4), (5, 7, 2, 0.5, 2), (100, 64, 33, 3.0, 6)])
def test_matches_oracle(lib, H, W, S, m, iters):
    """Ragged last cells, one-cell maps, the smallest S, several maps per
    launch, with and without masks and unusable pixels."""
    rng = np.random.default_rng(H * 31 + W * 7 + S)
    n = 3
    Ds = np.stack([_two_level(rng, H, W) for _ in range(n)])
    Ds[1].flat[rng.integers(0, Ds[1].size, max(1, Ds[1].size // 30))] = np.nan
    Ds[2].flat[rng.integers(0, Ds[2].size, max(1, Ds[2].size // 50))] = 5000.0
    Ms = (rng.random((n, H, W)) < 0.95).astype(np.uint8)
    got = lib.slic(_dev(Ds), S, m, iters)
    for i in range(n):
        _same([t[i] for t in got], Ds[i], S, m, iters)
    got = lib.slic(_dev(Ds), S, m, iters, mask=_dev(Ms))
    for i in range(n):
        _same([t[i] for t in got], Ds[i], S, m, iters, Ms[i])


def test_hand_worked_convergence(lib):
    """The stopping rule on the hand-worked maps: rounds at several
    tolerances and the unchanged result, as worked by hand."""
    import torch
    with open(os.path.join(GOLD, "hand_slic.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        D = np.array(c["disp"], np.float32)
        for tol, want in c["rounds_at_tol"]:
            r = torch.full((1,), -1, dtype=torch.int32, device="cuda")
            lab, d3, cen = lib.slic(_dev(D), c["S"], c["m"], 10, tol=tol, rounds=r)
            assert int(r[0]) == want, (c["note"][:30], tol)
            np.testing.assert_array_equal(lab.cpu().numpy()[0], c["labels"])
            np.testing.assert_array_equal(cen.cpu().numpy()[0], c["centres"])
            np.testing.assert_array_equal(d3.cpu().numpy()[0], c["d3"])


@pytest.mark.parametrize("tol", [0.0, 0.05, 0.3, 1.0])
def test_maps_stop_on_their_own_like_the_oracle(lib, tol):
    """Maps of one launch stop after different rounds (a flat map, a map
    that settles, noisy maps); each matches the oracle bit for bit with the
    same round count, with and without a mask."""
    import torch
    rng = np.random.default_rng(int(tol * 100) + 11)
    H, W, S, m = 48, 64, 8, 2.0
    Ds = np.stack([np.full((H, W), 3.0, np.float32)] + [_two_level(rng, H, W) for _ in range(3)])
    Ds[3] = np.round(Ds[3])  # two-valued steps settle sooner
    Ms = (rng.random(Ds.shape) < 0.9).astype(np.uint8)
    for mask in (None, Ms):
        r = torch.full((len(Ds),), -1, dtype=torch.int32, device="cuda")
        got = lib.slic(_dev(Ds), S, m, 30, mask=None if mask is None else _dev(mask), tol=tol, rounds=r)
        rounds = r.cpu().numpy()
        for i in range(len(Ds)):
            _same([t[i] for t in got], Ds[i], S, m, 30, None if mask is None else mask[i], tol=tol,
                  rounds=int(rounds[i]))
        assert rounds.min() < 30


def test_repeatable(lib):
    import torch
    rng = np.random.default_rng(3)
    D = _dev(np.stack([_two_level(rng, 200, 300) for _ in range(2)]))
    a = lib.slic(D, 12, 4.0, 8)
    b = lib.slic(D, 12, 4.0, 8)
    for x, y in zip(a, b):
        assert torch.equal(x.nan_to_num(-7.0) if x.is_floating_point() else x,
                          y.nan_to_num(-7.0) if y.is_floating_point() else y)


def test_full_size_batch_and_detection(lib):
    """16 maps of 1920 x 1080 in one launch (S = 16, at most 10 rounds,
    tol 0.25); one map against the oracle bit for bit with its round count;
    thresholding D3 finds the potholes with far fewer components than
    thresholding D2 pixel by pixel."""
    import torch
    rng = np.random.default_rng(8)
    n, H, W = 16, 1080, 1920
    Ds = np.stack([_two_level(rng, H, W, holes=2) for _ in range(n)])
    d = _dev(Ds)
    r = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    lab, d3, cen = lib.slic(d, 16, 4.0, 10, tol=0.25, rounds=r)
    _same([lab[7], d3[7], cen[7]], Ds[7], 16, 4.0, 10, tol=0.25, rounds=int(r[7]))
    assert ((r >= 1) & (r <= 10)).all()
    res, _ = lib.pothole_threshold(d, 0.0, 16.0, 128, 0.5)
    comps2 = lib.pothole_labels(d, res).cpu().numpy()
    comps3 = lib.pothole_labels(d3, res).cpu().numpy()
    for i in (0, 7):
        n2 = len(np.unique(comps2[i][comps2[i] > 0]))
        n3 = len(np.unique(comps3[i][comps3[i] > 0]))
        assert 0 < n3 <= n2
