"""The perspective-transformed path of the paper on one frame size, with the
road model estimated from the images themselves.

Every step is a HIP kernel behind the C ABI, enqueued on one stream with no
host synchronisation:
  1. 4 x 4 box reduction of both images;
  2. plain full-range SGM at quarter resolution (ndisp / 4 disparities);
  3. the road-model fit of Sec. II-C (eq. (11), (12)) on that coarse map,
     over pixels with disparity >= min_disp whose match lies at least
     `margin` coarse pixels inside the right image;
  4. per-row windows of `w` disparities at full resolution from the coarse
     fit (Sec. II-A: centred on the road line, or eq. (6) with delta_PT);
  5. SGM over those windows at full resolution: D1 in disparities of the
     original pair (eq. (10));
  6. the road model refitted on D1 and the disparity transformation of
     eq. (13): D2 = D1 - f(a, p, phi) + delta_DT.

The paper takes (a, phi) for the perspective transformation from its
Sec. II-C fit without saying which disparity map that fit runs on; here it
is the quarter-scale full-range result of the same frame, so the path needs
nothing but the two images.
"""
from __future__ import annotations

import torch

from . import sgm as S


class PerspectiveMatcher:
    """Frames of one size (W x H uint8 device images); see the module text.

    After match(): `coarse_fit` / `fit` are the device fits (sgm_road_fit
    records, float64 [1, 8]) of the quarter-scale map and of D1, `d_lo` the
    per-row window starts (int32 [H]) and `disp_int`, `disp_sub`, `d2` the
    outputs."""

    def __init__(self, width, height, ndisp=128, w=24, census=7, npaths=8, p1=10, p2=120, mode=0,
                 delta_pt=0.0, delta_dt=0.0, min_disp=0.5, margin=4.0, device=None):
        if width % 4 or height % 4:
            raise ValueError("width and height must be multiples of 4")
        self.W, self.H, self.w = int(width), int(height), int(w)
        self.mode, self.delta_pt, self.delta_dt = int(mode), float(delta_pt), float(delta_dt)
        self.min_disp, self.margin = float(min_disp), float(margin)
        self.device = torch.device(device or "cuda")
        Wc, Hc = self.W // 4, self.H // 4
        self.coarse = S.Matcher(Wc, Hc, census=census, ndisp=max(1, ndisp // 4), npaths=npaths, p1=p1, p2=p2,
                                device=self.device)
        self.fine = S.Matcher(self.W, self.H, census=census, ndisp=self.w, npaths=npaths, p1=p1, p2=p2,
                              device=self.device)
        dev = self.device
        self.left_c = torch.empty((Hc, Wc), dtype=torch.uint8, device=dev)
        self.right_c = torch.empty_like(self.left_c)
        self.coarse_int = torch.empty((Hc, Wc), dtype=torch.int16, device=dev)
        self.coarse_sub = torch.empty((Hc, Wc), dtype=torch.float32, device=dev)
        self.coarse_fit = torch.empty((1, S.ROAD_FIT_WORDS), dtype=torch.float64, device=dev)
        self.fit = torch.empty_like(self.coarse_fit)
        self.ws = torch.empty(max(S.road_workspace_size(self.W, self.H, 1), S.road_workspace_size(Wc, Hc, 1)),
                              dtype=torch.uint8, device=dev)
        self.d_lo2 = torch.empty((1, self.H), dtype=torch.int32, device=dev)
        self.d_lo = self.d_lo2[0]
        self.disp_int = torch.empty((self.H, self.W), dtype=torch.int16, device=dev)
        self.disp_sub = torch.empty((self.H, self.W), dtype=torch.float32, device=dev)
        self.d2 = torch.empty_like(self.disp_sub)

    def match(self, left, right, stream=None):
        S.sgm_downsample4(left, self.left_c, stream=stream)
        S.sgm_downsample4(right, self.right_c, stream=stream)
        self.coarse.match(self.left_c, self.right_c, disp_int=self.coarse_int, disp_sub=self.coarse_sub,
                          stream=stream)
        S.road_fit(self.coarse_sub, None, self.min_disp, self.margin, fit=self.coarse_fit, workspace=self.ws,
                   stream=stream)
        S.road_window(self.coarse_fit, self.W, self.H, self.w, self.mode, self.delta_pt, scale=4.0,
                      d_lo=self.d_lo2, stream=stream)
        self.fine.match(left, right, d_lo=self.d_lo, disp_int=self.disp_int, disp_sub=self.disp_sub,
                        stream=stream)
        S.road_fit(self.disp_sub, None, 4 * self.min_disp, 4 * self.margin, fit=self.fit, workspace=self.ws,
                   stream=stream)
        S.disparity_transform(self.disp_sub, self.fit, self.delta_dt, out=self.d2, stream=stream)
        return self.disp_int, self.disp_sub, self.d2
