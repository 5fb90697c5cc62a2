"""Batched SGM (persistent aggregation over mixed-size pairs, graph capture,
autotuner) against the oracle and against the single-pair path."""
import numpy as np
import pytest

import oracle
from paper_2012_10802_amd import synth

pytestmark = pytest.mark.gpu

N, R, P1, P2 = 7, 8, 10, 120


@pytest.fixture(scope="module")
def sgm():
    import torch
    from paper_2012_10802_amd import sgm as mod
    assert torch.cuda.is_available()
    return mod


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rand_pair(W, H, seed, shift=4):
    rng = np.random.default_rng(seed)
    L = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
    Rm = np.clip(np.roll(L, -shift, axis=1).astype(int) + rng.integers(-3, 4, size=(H, W)),
                 0, 255).astype(np.uint8)
    return L, Rm


# (W, H, w, pitch, with row windows): every lane width, ragged sizes
SMALL = [(97, 61, 24, 97, True), (160, 120, 64, 160, False), (200, 150, 128, 256, False),
         (45, 33, 16, 45, True), (64, 40, 192, 64, False), (70, 9, 256, 80, False),
         (33, 70, 32, 33, False), (51, 47, 48, 64, True)]


def _small_batch(sgm, seed=0):
    pairs, host = [], []
    for i, (W, H, w, pitch, rows) in enumerate(SMALL):
        L, Rm = _rand_pair(pitch, H, 100 * seed + i)
        d_lo = (np.random.default_rng(i).integers(0, 5, size=H).astype(np.int32) if rows else None)
        pairs.append({"left": _dev(L), "right": _dev(Rm), "ndisp": w, "width": W,
                      "d_lo": None if d_lo is None else _dev(d_lo)})
        host.append((L[:, :W], Rm[:, :W], w, d_lo))
    return pairs, host


def _check_against_oracle(b, host):
    for i, (L, Rm, w, d_lo) in enumerate(host):
        want_i, want_s = oracle.sgm(L, Rm, N, w, R, P1, P2, d_lo)
        got_i = b.disp_int[i].cpu().numpy().view(np.uint16)
        np.testing.assert_array_equal(got_i, want_i, err_msg="pair %d" % i)
        np.testing.assert_array_equal(b.disp_sub[i].cpu().numpy(), want_s, err_msg="pair %d" % i)


def test_small_mixed_batch_matches_oracle(sgm):
    import torch
    pairs, host = _small_batch(sgm)
    b = sgm.Batch(pairs, census=N, npaths=R, p1=P1, p2=P2)
    b.run()
    torch.cuda.synchronize()
    _check_against_oracle(b, host)


@pytest.mark.parametrize("tuning", [(1, 0, 0), (4, 1, 16), (32, 2, 8), (8, 0, 4), (8, 0, 16), (12, 2, 0)])
def test_every_tuning_gives_identical_results(sgm, tuning):
    """Waves per CU, queue order and lanes per scanline (0: the default
    mapping of each width; 4 and 8 apply to the widths they serve, the
    others keep 16) change nothing in the results."""
    import torch
    pairs, host = _small_batch(sgm, seed=1)
    b = sgm.Batch(pairs, census=N, npaths=R, p1=P1, p2=P2)
    b.tuning = tuning
    assert b.tuning == tuning
    b.run()
    torch.cuda.synchronize()
    _check_against_oracle(b, host)


def test_graph_replays_follow_new_inputs(sgm):
    """Capture once, then replay with different images copied into the same
    input buffers, with eager work in between; every replay must match the
    oracle on the inputs it saw."""
    import torch
    pairs, host = _small_batch(sgm, seed=2)
    b = sgm.Batch(pairs, census=N, npaths=R, p1=P1, p2=P2)
    s = torch.cuda.Stream()
    b.capture(s)
    for rep in range(3):
        if rep:
            host = []
            for i, (W, H, w, pitch, rows) in enumerate(SMALL):
                L, Rm = _rand_pair(pitch, H, 1000 * rep + i, shift=3 + rep)
                pairs[i]["left"].copy_(_dev(L))
                pairs[i]["right"].copy_(_dev(Rm))
                d_lo = (pairs[i]["d_lo"].cpu().numpy() if rows else None)
                host.append((L[:, :W], Rm[:, :W], w, d_lo))
            # unrelated eager work on the default stream between replays
            m = sgm.Matcher(64, 32, census=5, ndisp=32, npaths=4)
            m.match(pairs[0]["left"][:32, :64].contiguous(), pairs[0]["right"][:32, :64].contiguous())
        torch.cuda.synchronize()
        b.launch(s)
        s.synchronize()
        _check_against_oracle(b, host)


def test_autotune_cache(sgm, tmp_path):
    import torch
    pairs, host = _small_batch(sgm, seed=3)
    b = sgm.Batch(pairs, census=N, npaths=R, p1=P1, p2=P2)
    cache = tmp_path / "tune.txt"
    t1 = b.autotune(cache)
    assert cache.exists() and len(cache.read_text().splitlines()) == 1
    b2 = sgm.Batch(pairs, census=N, npaths=R, p1=P1, p2=P2)
    assert b2.autotune(cache) == t1  # read back, no new line
    assert len(cache.read_text().splitlines()) == 1
    bad = tmp_path / "corrupt.txt"
    bad.write_bytes(b"\x00\xff garbage\nnot a line\n")
    b3 = sgm.Batch(pairs, census=N, npaths=R, p1=P1, p2=P2)
    b3.autotune(bad)
    b3.run()
    torch.cuda.synchronize()
    _check_against_oracle(b3, host)


def _road_workload(counts, seed0=4000, unique=2):
    """Pairs of the 64-pair mixed workload: `counts` maps a road config to a
    number of pairs; `unique` distinct renders per size are reused."""
    out = []
    for name, cnt in counts:
        c = synth.CONFIGS[name]
        renders = [synth.make_pair(synth.scene_for_config(name, seed0 + k), seed0 + k)
                   for k in range(min(unique, cnt))]
        for j in range(cnt):
            out.append((name, c["ndisp"], renders[j % len(renders)]))
    return out


@pytest.fixture(scope="module")
def mixed64(sgm):
    """The 64-pair mixed workload (24 x 640x480 w 64, 24 x 1280x720 w 128,
    16 x 1920x1080 w 192) run once as one batch."""
    import torch
    work = _road_workload([("road640", 24), ("road1280", 24), ("road1920", 16)])
    dev_imgs = {}
    pairs = []
    for name, w, p in work:
        key = id(p)
        if key not in dev_imgs:
            dev_imgs[key] = (_dev(p.left), _dev(p.right))
        L, Rm = dev_imgs[key]
        pairs.append({"left": L, "right": Rm, "ndisp": w})
    b = sgm.Batch(pairs, census=N, npaths=R, p1=P1, p2=P2)
    b.run()
    torch.cuda.synchronize()
    out = [(b.disp_int[i].cpu().numpy(), b.disp_sub[i].cpu().numpy()) for i in range(len(work))]
    del b, pairs
    torch.cuda.empty_cache()
    return work, dev_imgs, out


def test_mixed_64_pair_workload_matches_single_pair_path(sgm, mixed64):
    """Every pair of the 64-pair batch equals sgm_match on that pair."""
    import torch
    work, dev_imgs, out = mixed64
    singles = {}
    for i, (name, w, p) in enumerate(work):
        key = id(p)
        if key not in singles:
            H, W = p.left.shape
            m = sgm.Matcher(W, H, census=N, ndisp=w, npaths=R, p1=P1, p2=P2)
            di, ds = m.match(*dev_imgs[key])
            torch.cuda.synchronize()
            singles[key] = (di.cpu().numpy(), ds.cpu().numpy())
            del m
        np.testing.assert_array_equal(out[i][0], singles[key][0], err_msg="pair %d" % i)
        np.testing.assert_array_equal(out[i][1], singles[key][1], err_msg="pair %d" % i)


@pytest.mark.parametrize("size", ["road640", "road1280", "road1920"])
def test_mixed_64_pair_workload_matches_oracle(mixed64, size):
    """One pair of each size of the 64-pair batch equals the oracle over the
    whole frame: integer disparity bit for bit, sub-pixel disparity within
    1e-4 px (and in fact bit for bit)."""
    work, _, out = mixed64
    i = next(k for k, (name, _, _) in enumerate(work) if name == size)
    name, w, p = work[i]
    want_i, want_s = oracle.sgm(p.left, p.right, N, w, R, P1, P2)
    got_i = out[i][0].view(np.uint16)
    np.testing.assert_array_equal(got_i, want_i, err_msg="pair %d (%s)" % (i, name))
    assert np.abs(out[i][1] - want_s).max() <= 1e-4
    np.testing.assert_array_equal(out[i][1], want_s, err_msg="pair %d (%s)" % (i, name))
