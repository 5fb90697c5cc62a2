"""The perspective-transformed path of the paper on batches of frames of one
size, with the road model estimated from the images themselves.

Every step is a HIP kernel behind the C ABI, each covering the whole batch,
enqueued on one stream with no host synchronisation:
  1. 4 x 4 box reduction of both images;
  2. plain full-range SGM at quarter resolution (ndisp / 4 disparities);
  3. the road-model fit of Sec. II-C (eq. (11), (12)) on each coarse map,
     over pixels with disparity >= min_disp whose match lies at least
     `margin` coarse pixels inside the right image, refitted over the
     pixels within `coarse_tols` of the previous fit's road line;
  4. search windows at full resolution from the coarse fits:
       windows="pixel" (default): 16 disparities per pixel centred on the
         fitted road plane, which carries the roll of eq. (3) along each
         row as well as the pitch down the image;
       windows="row": `w` disparities per row (Sec. II-A: centred on the
         road line at the row centre, or eq. (6) with delta_PT);
  5. SGM over those windows at full resolution: D1 in disparities of the
     original pair (eq. (10));
  6. the road model refitted on D1 (over the pixels within `fine_tols` of
     the previous fit) and the disparity transformation of eq. (13):
     D2 = D1 - f(a, p, phi) + delta_DT.

The paper takes (a, phi) for the perspective transformation from its
Sec. II-C fit without saying which disparity map that fit runs on; here it
is the quarter-scale full-range result of the same frame, so the path needs
nothing but the two images.
"""
from __future__ import annotations

import torch

from . import sgm as S

PIXEL_WINDOW = 16  # width of the per-pixel windows (the windowed kernels' width)


class PerspectiveMatcher:
    """Batches of `batch` frames (W x H uint8 device images, [batch, H, W],
    or [H, W] when batch is 1); see the module text.

    After match(): `coarse_fits` / `fits` are the device fits (sgm_road_fit
    records, float64 [batch, 8]) of the quarter-scale maps and of D1, first
    fit then refits (`coarse_fit`, `fit` the last of each); `lo` the
    per-pixel window starts (int32 [batch, H, W], windows="pixel") or `d_lo`
    the per-row ones (int32 [batch, H], windows="row"); `disp_int`,
    `disp_sub`, `d2` the outputs [batch, H, W]."""

    def __init__(self, width, height, batch=1, ndisp=128, w=24, census=7, npaths=8, p1=10, p2=120,
                 windows="pixel", mode=0, delta_pt=0.0, delta_dt=0.0, min_disp=0.5, margin=4.0,
                 coarse_tols=(1.0,), fine_tols=(2.0, 1.0), autotune=True, device=None):
        if width % 4 or height % 4:
            raise ValueError("width and height must be multiples of 4")
        if windows not in ("pixel", "row"):
            raise ValueError("windows must be 'pixel' or 'row'")
        self.W, self.H, self.n = int(width), int(height), int(batch)
        self.windows = windows
        self.w = PIXEL_WINDOW if windows == "pixel" else int(w)
        self.mode, self.delta_pt, self.delta_dt = int(mode), float(delta_pt), float(delta_dt)
        self.min_disp, self.margin = float(min_disp), float(margin)
        self.coarse_tols = tuple(float(t) for t in coarse_tols)
        self.fine_tols = tuple(float(t) for t in fine_tols)
        self.device = dev = torch.device(device or "cuda")
        n, H, W = self.n, self.H, self.W
        Wc, Hc = W // 4, H // 4
        self.left_c = torch.empty((n, Hc, Wc), dtype=torch.uint8, device=dev)
        self.right_c = torch.empty_like(self.left_c)
        self.coarse_int = torch.empty((n, Hc, Wc), dtype=torch.int16, device=dev)
        self.coarse_sub = torch.empty((n, Hc, Wc), dtype=torch.float32, device=dev)
        self.coarse = S.Batch([dict(left=self.left_c[i], right=self.right_c[i], ndisp=max(1, ndisp // 4),
                                    disp_int=self.coarse_int[i], disp_sub=self.coarse_sub[i]) for i in range(n)],
                              census=census, npaths=npaths, p1=p1, p2=p2, device=dev)
        fit = lambda: torch.empty((n, S.ROAD_FIT_WORDS), dtype=torch.float64, device=dev)  # noqa: E731
        self.coarse_fits = [fit() for _ in range(1 + len(self.coarse_tols))]
        self.fits = [fit() for _ in range(1 + len(self.fine_tols))]
        self.coarse_fit, self.fit = self.coarse_fits[-1], self.fits[-1]
        self.ws = torch.empty(max(S.road_workspace_size(W, H, n), S.road_workspace_size(Wc, Hc, n)),
                              dtype=torch.uint8, device=dev)
        self.disp_int = torch.empty((n, H, W), dtype=torch.int16, device=dev)
        self.disp_sub = torch.empty((n, H, W), dtype=torch.float32, device=dev)
        self.d2 = torch.empty_like(self.disp_sub)
        if windows == "pixel":
            self.fine = S.Matcher(W, H, census=census, ndisp=self.w, npaths=npaths, p1=p1, p2=p2, device=dev)
            self.lo = torch.empty((n, H, W), dtype=torch.int32, device=dev)
            self.win_ws = self.fine.win_batch_workspace(n)
        else:
            self.left_f = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
            self.right_f = torch.empty_like(self.left_f)
            self.d_lo = torch.empty((n, H), dtype=torch.int32, device=dev)
            self.fine = S.Batch([dict(left=self.left_f[i], right=self.right_f[i], ndisp=self.w, d_lo=self.d_lo[i],
                                      disp_int=self.disp_int[i], disp_sub=self.disp_sub[i]) for i in range(n)],
                                census=census, npaths=npaths, p1=p1, p2=p2, device=dev)
        if autotune:
            # launch shapes of the batched stages (lane mapping, waves per CU,
            # queue order), timed once on these buffers
            self.left_c.zero_()
            self.right_c.zero_()
            self.coarse.autotune()
            if windows == "row":
                self.left_f.zero_()
                self.right_f.zero_()
                self.d_lo.zero_()
                self.fine.autotune()

    def _fit(self, disp, fits, tols, min_disp, margin, stream):
        S.road_fit(disp, None, min_disp, margin, fit=fits[0], workspace=self.ws, stream=stream)
        for i, tol in enumerate(tols):
            S.road_fit(disp, None, min_disp, margin, prior=fits[i], tol=tol, fit=fits[i + 1], workspace=self.ws,
                       stream=stream)

    def match(self, left, right, stream=None, refit=True):
        """Steps 1-6 (refit=False: steps 1-5 only, for a caller that fits
        D1 itself; `fits` and `d2` are then left as they were and d2 is
        returned as None)."""
        if left.dim() == 2:
            left, right = left.unsqueeze(0), right.unsqueeze(0)
        if tuple(left.shape) != (self.n, self.H, self.W) or left.shape != right.shape:
            raise ValueError("left and right must be uint8 [batch, H, W]")
        S.sgm_downsample4_batch(left, self.left_c, stream=stream)
        S.sgm_downsample4_batch(right, self.right_c, stream=stream)
        self.coarse.run(stream=stream)
        self._fit(self.coarse_sub, self.coarse_fits, self.coarse_tols, self.min_disp, self.margin, stream)
        if self.windows == "pixel":
            S.road_window_map(self.coarse_fit, self.W, self.H, self.w, scale=4.0, lo=self.lo, stream=stream)
            self.fine.match_win_batch(left, right, self.lo, disp_int=self.disp_int, disp_sub=self.disp_sub,
                                      workspace=self.win_ws, stream=stream)
        else:
            S.road_window(self.coarse_fit, self.W, self.H, self.w, self.mode, self.delta_pt, scale=4.0,
                          d_lo=self.d_lo, stream=stream)
            with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
                self.left_f.copy_(left)  # the batch reads its own input buffers
                self.right_f.copy_(right)
            self.fine.run(stream=stream)
        if not refit:
            return self.disp_int, self.disp_sub, None
        self._fit(self.disp_sub, self.fits, self.fine_tols, 4 * self.min_disp, 4 * self.margin, stream)
        S.disparity_transform(self.disp_sub, self.fit, self.delta_dt, out=self.d2, stream=stream)
        return self.disp_int, self.disp_sub, self.d2
