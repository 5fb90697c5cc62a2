"""sgm_match_noalloc (the whole path with the library's own scratch array)
against sgm_match with a caller workspace, called through the C ABI: two
calls in a row on one device, the second on a smaller frame, every output
bit for bit."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2012_10802_amd import sgm, synth

pytestmark = pytest.mark.gpu

# (workload recipe, seed, width, height, census, ndisp, npaths, d_lo from the road model)
CASES = [("road320", 11, 320, 240, 5, 32, 4, False),
         ("road320", 12, 200, 150, 7, 24, 8, True)]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _pair(name, seed, W, H):
    p = synth.make_pair(synth.scene_for_config(name, seed), seed)
    return p, np.ascontiguousarray(p.left[:H, :W]), np.ascontiguousarray(p.right[:H, :W])


def test_noalloc_matches_match_twice_second_smaller():
    lib = sgm.library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream(dev)
    for name, seed, W, H, n, w, R, with_dlo in CASES:
        print("noalloc case %dx%dx%d census %d paths %d" % (W, H, w, n, R), flush=True)
        p, left, right = _pair(name, seed, W, H)
        L = torch.from_numpy(left).to(dev)
        Rt = torch.from_numpy(right).to(dev)
        d_lo = None
        if with_dlo:
            a0, a1, phi = p.road_params
            d_lo = sgm.sgm_window_from_road(a0, a1, phi, W, H, w, mode=0).to(dev)
        plan = sgm.sgm_plan(W, H, n, w, R, 10, 120)
        try:
            need = sgm.sgm_workspace_size(plan)
            assert need <= 64 << 20
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
            outs = []
            for call in ("sgm_match", "sgm_match_noalloc"):
                di = torch.full((H, W), -1, dtype=torch.int16, device=dev)
                ds = torch.full((H, W), float("nan"), dtype=torch.float32, device=dev)
                if call == "sgm_match":
                    st = lib.sgm_match(plan, _ptr(L), _ptr(Rt), W, _ptr(d_lo), _ptr(di), _ptr(ds), _ptr(ws),
                                       need, ctypes.c_void_p(stream.cuda_stream))
                else:
                    st = lib.sgm_match_noalloc(plan, _ptr(L), _ptr(Rt), W, _ptr(d_lo), _ptr(di), _ptr(ds),
                                               ctypes.c_void_p(stream.cuda_stream))
                assert st == 0, lib.sgm_last_error()
                torch.cuda.synchronize()
                outs.append((di.cpu().numpy(), ds.cpu().numpy()))
            (ri, rs), (gi, gs) = outs
            assert np.array_equal(ri, gi)
            assert np.array_equal(rs.view(np.uint32), gs.view(np.uint32))
            assert (gi >= 0).all()
        finally:
            sgm.sgm_plan_free(plan)
