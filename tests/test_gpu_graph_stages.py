"""The stages after matching (road fit, windows, eq. (13), pothole
threshold and labels, SLIC and D3) captured once in a HIP graph through
torch, replayed on new inputs copied into the captured buffers, with eager
work in between: every replay equals an eager run on the same inputs (the
calls allocate nothing and clear their scratch with kernels, so they can be
captured)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _maps(seed, n, H, W):
    rng = np.random.default_rng(seed)
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    out = []
    for i in range(n):
        phi = math.radians(rng.uniform(-3, 3))
        D = 20 + 0.1 * (math.cos(phi) * (v - (H - 1) / 2) - math.sin(phi) * (u - (W - 1) / 2))
        cu, cv = rng.uniform(40, W - 40), rng.uniform(40, H - 40)
        r2 = ((u - cu) / 30) ** 2 + ((v - cv) / 20) ** 2
        D = np.where(r2 < 1, D - 3 * (1 - r2), D) + rng.normal(0, 0.2, (H, W))
        out.append(D)
    return np.stack(out).astype(np.float32)


def test_post_matching_stages_replay_in_a_graph():
    import torch
    from paper_2012_10802_amd import sgm
    n, H, W = 2, 240, 320
    dev = torch.device("cuda")
    D = torch.from_numpy(_maps(1, n, H, W)).to(dev)
    mask = torch.ones((n, H, W), dtype=torch.uint8, device=dev)
    mask[:, :, :8] = 0
    fit = torch.empty((n, sgm.ROAD_FIT_WORDS), dtype=torch.float64, device=dev)
    fws = torch.empty(sgm.road_workspace_size(W, H, n), dtype=torch.uint8, device=dev)
    d_lo = torch.empty((n, H), dtype=torch.int32, device=dev)
    d2 = torch.empty_like(D)
    res = torch.empty((n, sgm.POTHOLE_WORDS), dtype=torch.float64, device=dev)
    pws = torch.empty(sgm.pothole_workspace_size(64, n), dtype=torch.uint8, device=dev)
    lab = torch.empty((n, H, W), dtype=torch.int32, device=dev)
    sl = torch.empty_like(lab)
    d3 = torch.empty_like(D)
    cen = torch.empty((n, sgm.slic_num_centres(W, H, 8), 3), dtype=torch.float64, device=dev)
    sws = torch.empty(sgm.slic_workspace_size(W, H, 8, n), dtype=torch.uint8, device=dev)

    def chain():
        sgm.road_fit(D, mask, 0.5, 2.0, fit=fit, workspace=fws)
        sgm.road_window(fit, W, H, 24, 1, 2.0, d_lo=d_lo)
        sgm.disparity_transform(D, fit, 10.0, out=d2)
        sgm.pothole_threshold(d2, 2.0, 18.0, 64, 0.5, mask=mask, result=res, workspace=pws)
        sgm.pothole_labels(d2, res, mask=mask, labels=lab)
        sgm.slic(d2, 8, 4.0, 4, mask=mask, labels=sl, d3=d3, centres=cen, workspace=sws)

    def outputs():
        return [t.clone() for t in (fit, d_lo, d2, res, lab, sl, d3, cen)]

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        chain()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        chain()
    for rep in range(3):
        D.copy_(torch.from_numpy(_maps(10 + rep, n, H, W)).to(dev))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = outputs()
        chain()  # eager, same inputs and buffers
        torch.cuda.synchronize()
        want = outputs()
        for name, a, b in zip(("fit", "d_lo", "d2", "res", "lab", "sl", "d3", "cen"), got, want):
            if name == "res":  # E2 is a float64 atomic sum: its last bits may differ
                ga, wa = sgm.pothole_threshold_dicts(a), sgm.pothole_threshold_dicts(b)
                for x, y in zip(ga, wa):
                    assert (x["k"], x["n1"], x["n2"], x["t_s"]) == (y["k"], y["n1"], y["n2"], y["t_s"])
                    assert x["e2"] == pytest.approx(y["e2"], rel=1e-9)
            else:
                assert torch.equal(a.nan_to_num(-1.0) if a.is_floating_point() else a,
                                   b.nan_to_num(-1.0) if b.is_floating_point() else b), (rep, name)
        assert sgm.road_fit_dicts(got[0])[0]["status"] == 0
