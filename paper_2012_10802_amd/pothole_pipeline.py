"""Stereo pairs to labelled potholes: the whole method of the paper on a
batch of pairs of one size, every step a HIP kernel behind the C ABI,
enqueued on one stream (the learned-window matcher adds its side streams).

  1. disparity D1 (Sec. II-A, II-B): the perspective-transformed path (the
     default: quarter-scale SGM, road fit, per-pixel windows on the fitted
     road plane, windowed SGM; road_pipeline.PerspectiveMatcher), the
     learned-window SGM, or plain full-range batched SGM;
  2. road model (Sec. II-C, eq. (11), (12)) fitted to D1 over the pixels
     with d >= min_disp whose match lies `margin` pixels inside the right
     image, then refitted over the pixels within each of `refit_tols` of the
     previous fit's road line (the road disparities; the first fit is pulled
     by the background near the horizon and other outliers);
  3. the road region (road disparity f >= f_min: below the fitted horizon
     line, and u - f >= margin: right of the band where the road cannot be
     matched; the paper selects its road regions by hand) and the
     transformed map D2 = D1 - f + delta_DT (eq. (13));
  4. the threshold t_r of eq. (14), (15) from D2's vectors over the road
     region, on `nbins` bins spanning delta_DT +- span, and
     t_s = t_r - delta_PD;
  5. SLIC superpixels on D2 over the road region (Sec. II-D), at most
     `slic_iters` rounds, each map stopping once its largest centre change
     is within `slic_tol` (the residual of Sec. II-D), and their means D3
     (Sec. II-E);
  6. potholes: the 8-connected components of D3 below t_s, labelled
     1 + the smallest row-major index of the component; with
     `prune_single` (default) those lying in a single superpixel are
     removed, as Sec. III-B counts them as false detections.
"""
from __future__ import annotations

import torch

from . import sgm as S

# SLIC stops once no centre moves by more than this (in disparities, with
# the spatial part weighted by (m / S)^2) in one round
SLIC_TOL = 0.25


class PotholeDetector:
    """detect(left, right) on uint8 device stacks [batch, H, W]; returns the
    pothole labels int32 [batch, H, W].  Intermediate maps stay available
    as attributes: disp (D1), fit, road, d2, threshold, superpixels, d3,
    slic_rounds (the SLIC rounds each map ran)."""

    def __init__(self, width, height, batch, ndisp=192, census=7, npaths=8, p1=10, p2=120, matcher="perspective",
                 net=None, delta_dt=10.0, delta_pd=0.5, nbins=128, span=8.0, slic_step=16, slic_m=4.0,
                 slic_iters=10, slic_tol=SLIC_TOL, min_disp=0.5, margin=4.0, f_min=2.0, refit_tols=(2.0, 1.0),
                 prune_single=True, device="cuda"):
        self.W, self.H, self.n = int(width), int(height), int(batch)
        self.delta_dt, self.delta_pd, self.nbins, self.span = float(delta_dt), float(delta_pd), int(nbins), span
        self.slic_step, self.slic_m, self.slic_iters = int(slic_step), float(slic_m), int(slic_iters)
        self.slic_tol = float(slic_tol)
        self.min_disp, self.margin, self.f_min = float(min_disp), float(margin), float(f_min)
        self.refit_tols = tuple(float(t) for t in refit_tols)
        self.prune_single = bool(prune_single)
        dev = self.device = torch.device(device)
        n, H, W = self.n, self.H, self.W
        if matcher == "perspective":
            from .road_pipeline import PerspectiveMatcher
            self.matcher = PerspectiveMatcher(W, H, batch=n, ndisp=ndisp, census=census, npaths=npaths, p1=p1,
                                              p2=p2, windows="pixel", delta_dt=delta_dt, device=device)
            self._match = self._match_perspective
        elif matcher == "learned":
            from .learned_window import LearnedWindowMatcher
            self.matcher = LearnedWindowMatcher(W, H, batch=n, ndisp=ndisp, census=census, npaths=npaths, p1=p1,
                                                p2=p2, net=net, device=device)
            self._match = self.matcher.match
        elif matcher == "plain":
            self._left = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
            self._right = torch.empty_like(self._left)
            self._dint = torch.empty((n, H, W), dtype=torch.int16, device=dev)
            self._dsub = torch.empty((n, H, W), dtype=torch.float32, device=dev)
            self.matcher = S.Batch([dict(left=self._left[i], right=self._right[i], ndisp=ndisp,
                                         disp_int=self._dint[i], disp_sub=self._dsub[i]) for i in range(n)],
                                   census=census, npaths=npaths, p1=p1, p2=p2, device=dev)
            self._match = self._match_plain
        else:
            raise ValueError("matcher must be 'perspective', 'learned' or 'plain'")
        # fits[0] the first fit, fits[i] the refit with refit_tols[i - 1]; fit the last
        self.fits = [torch.empty((n, S.ROAD_FIT_WORDS), dtype=torch.float64, device=dev)
                     for _ in range(1 + len(self.refit_tols))]
        self.fit = self.fits[-1]
        self.fit_ws = torch.empty(S.road_workspace_size(W, H, n), dtype=torch.uint8, device=dev)
        self.road = torch.empty((n, H, W), dtype=torch.uint8, device=dev)
        self.d2 = torch.empty((n, H, W), dtype=torch.float32, device=dev)
        self.threshold = torch.empty((n, S.POTHOLE_WORDS), dtype=torch.float64, device=dev)
        self.thr_ws = torch.empty(S.pothole_workspace_size(self.nbins, n), dtype=torch.uint8, device=dev)
        self.superpixels = torch.empty((n, H, W), dtype=torch.int32, device=dev)
        self.d3 = torch.empty_like(self.d2)
        self.centres = torch.empty((n, S.slic_num_centres(W, H, self.slic_step), 3), dtype=torch.float64,
                                   device=dev)
        self.slic_ws = torch.empty(S.slic_workspace_size(W, H, self.slic_step, n), dtype=torch.uint8, device=dev)
        self.slic_rounds = torch.empty((n,), dtype=torch.int32, device=dev)
        self.labels = torch.empty((n, H, W), dtype=torch.int32, device=dev)
        self.disp = None

    def _match_perspective(self, left, right, stream=None):
        # the detector fits D1 itself (step 2), so the matcher stops at D1
        dint, dsub, _ = self.matcher.match(left, right, stream=stream, refit=False)
        return dint, dsub

    def _match_plain(self, left, right, stream=None):
        with torch.cuda.stream(stream if stream is not None else torch.cuda.current_stream()):
            self._left.copy_(left)  # the batch reads its own input buffers
            self._right.copy_(right)
        self.matcher.run(stream=stream)
        return self._dint, self._dsub

    def detect(self, left, right, stream=None):
        _, d1 = self._match(left, right, stream=stream)
        self.disp = d1
        S.road_fit(d1, None, self.min_disp, self.margin, fit=self.fits[0], workspace=self.fit_ws, stream=stream)
        for i, tol in enumerate(self.refit_tols):
            S.road_fit(d1, None, self.min_disp, self.margin, prior=self.fits[i], tol=tol, fit=self.fits[i + 1],
                       workspace=self.fit_ws, stream=stream)
        S.road_mask(d1, self.fit, self.f_min, self.margin, mask=self.road, stream=stream)
        S.disparity_transform(d1, self.fit, self.delta_dt, out=self.d2, stream=stream)
        S.pothole_threshold(self.d2, self.delta_dt - self.span, self.delta_dt + self.span, self.nbins,
                            self.delta_pd, mask=self.road, result=self.threshold, workspace=self.thr_ws,
                            stream=stream)
        S.slic(self.d2, self.slic_step, self.slic_m, self.slic_iters, mask=self.road, tol=self.slic_tol,
               labels=self.superpixels, d3=self.d3, centres=self.centres, workspace=self.slic_ws,
               rounds=self.slic_rounds, stream=stream)
        S.pothole_labels(self.d3, self.threshold, mask=self.road, labels=self.labels, stream=stream)
        if self.prune_single:
            S.pothole_prune(self.labels, self.superpixels, stream=stream)
        return self.labels
