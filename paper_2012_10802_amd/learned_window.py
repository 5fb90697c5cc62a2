"""Learned search windows (the learned-window form of the SGM path).

Pipeline for a batch of pairs of one size, every step a HIP kernel behind
the C ABI:
  1. 4 x 4 box reduction of both images (quarter resolution);
  2. plain full-range SGM of all quarter-resolution pairs (ndisp / 4
     disparities) in one batched launch: the coarse disparity;
  3. the window network (four 3x3 convolutions, 16 channels, bfloat16 on
     the matrix cores) on [coarse disparity, coarse left image, distance of
     the coarse match from the left border]: a centre offset and a
     confidence logit per coarse pixel;
  4. the window map: per full-resolution pixel a 16-wide window centred on
     4 * (coarse + offset) where the network is confident; the other pixels
     are marked for the fallback (their window, centred on 4 * coarse, still
     feeds the windowed aggregation of their neighbours);
  5. SGM over the per-pixel windows at full resolution, every pair of the
     batch in one set of launches;
  6. the full-range fallback: plain SGM over all ndisp disparities on
     rectangles around the marked pixels (on a side stream that starts once
     the window maps are known and runs beside step 5) (their rows and columns widened by
     a margin, and by ndisp - 1 more columns to the left so that every
     disparity finds its right-image pixel; the whole frame once they cover
     most of it), whose result replaces the windowed one on the marked
     pixels.  With every pixel marked the output is plain full-range SGM of
     the frame, exactly.

The network is the project's own addition: the paper's windows come from
its road model (Sec. II-A, eq. (3) and (6)) one per row; here a window is
predicted per pixel from the quarter-scale SGM result.

Training (train_window.py): pairs from the road generator, labelled by
full-range plain SGM at full resolution on the GPU; Adam on float32 master
weights with the hand-written forward, loss, backward and optimiser
kernels.  Checkpoints are plain arrays (numpy .npz, no pickles) with a JSON
header.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np
import torch

from . import sgm as S

CH = 16
OUT_CH = 2  # network outputs kept: centre offset, confidence logit
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "window_cnn.npz")
_lib = S.library()


def _c(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def num_params() -> int:
    return int(_lib.sgm_cnn_num_params())


def init_params(seed=0):
    """He-normal weights on the used input channels (three in the first
    layer), zero biases; the last layer starts small."""
    rng = np.random.default_rng(seed)
    per = 9 * CH * CH + CH
    p = np.zeros(4 * per, np.float32)
    for l in range(4):
        fan_in = 9 * (3 if l == 0 else CH)
        Wl = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(9, CH, CH)).astype(np.float32)
        if l == 0:
            Wl[:, :, 3:] = 0.0
        if l == 3:
            Wl *= 0.1
        p[l * per: l * per + 9 * CH * CH] = Wl.ravel()
    return p


class WindowNet:
    """Parameters, Adam moments and bfloat16 weight layouts of the network."""

    def __init__(self, params=None, seed=0, device="cuda"):
        self.device = torch.device(device)
        if params is None:
            params = init_params(seed)
        params = np.ascontiguousarray(params, np.float32)
        if params.shape != (num_params(),):
            raise ValueError("expected %d parameters" % num_params())
        self.params = torch.from_numpy(params.copy()).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step = 0
        self.header = {}
        self.wf = torch.empty(4 * 9 * CH * CH, dtype=torch.int16, device=self.device)
        self.wb = torch.empty_like(self.wf)
        self.pack()

    def pack(self):
        S._check(_lib.sgm_cnn_pack_weights(_c(self.params), _c(self.wf), _c(self.wb), S._stream()),
                 "sgm_cnn_pack_weights")

    # --- buffers for n images of W x H
    def buffers(self, W, H, n):
        act = torch.empty((3, n, H, W, CH), dtype=torch.int16, device=self.device)
        out = torch.empty((n, H, W, OUT_CH), dtype=torch.float32, device=self.device)
        return act, out

    def forward(self, x0, acts, out, W, H, n, stream=None):
        S._check(_lib.sgm_cnn_forward(_c(self.wf), _c(self.params), _c(x0), W, H, n, _c(acts), _c(out),
                                      S._stream(stream)), "sgm_cnn_forward")
        return out

    def infer(self, x0, out, W, H, n, stream=None):
        """forward without hidden activations (one launch; same out)"""
        S._check(_lib.sgm_cnn_infer(_c(self.wf), _c(self.params), _c(x0), W, H, n, _c(out), S._stream(stream)),
                 "sgm_cnn_infer")
        return out

    def train_buffers(self, W, H, n):
        acts, out = self.buffers(W, H, n)
        dy = torch.empty((n, H, W, CH), dtype=torch.int16, device=self.device)
        scratch = torch.empty(int(_lib.sgm_cnn_scratch_bytes(W, H, n)), dtype=torch.uint8,
                              device=self.device)
        loss = torch.zeros(2, dtype=torch.float32, device=self.device)
        return acts, out, dy, scratch, loss

    def train_step(self, x0, coarse, label, W, H, n, lr, bufs, stream=None):
        """Forward, loss, backward, Adam.  Returns the device loss pair
        (offset term, confidence term) without synchronising."""
        acts, out, dy, scratch, loss = bufs
        st = S._stream(stream)
        self.forward(x0, acts, out, W, H, n, stream)
        loss.zero_()
        S._check(_lib.sgm_cnn_loss(_c(out), _c(coarse), _c(label), W, H, n, _c(dy), _c(loss), st),
                 "sgm_cnn_loss")
        S._check(_lib.sgm_cnn_backward(_c(self.wb), _c(x0), _c(acts), _c(dy), W, H, n, _c(self.grad),
                                       _c(scratch), scratch.numel(), st), "sgm_cnn_backward")
        self.step += 1
        S._check(_lib.sgm_cnn_adam(_c(self.params), _c(self.m), _c(self.v), _c(self.grad), self.step,
                                   float(lr), 0.9, 0.999, 1e-8, _c(self.wf), _c(self.wb), st), "sgm_cnn_adam")
        return loss

    # --- checkpoints: plain arrays + JSON header (no pickles)
    def save(self, path, extra=None):
        header = {"format": "window-cnn/1", "step": self.step, "num_params": num_params()}
        header.update(extra or {})
        tmp = path + ".tmp.npz"
        np.savez(tmp, params=self.params.cpu().numpy(), m=self.m.cpu().numpy(),
                 v=self.v.cpu().numpy(),
                 header=np.frombuffer(json.dumps(header).encode(), dtype=np.uint8))
        os.replace(tmp, path)

    @classmethod
    def load(cls, path, device="cuda"):
        with np.load(path, allow_pickle=False) as z:
            header = json.loads(bytes(z["header"]).decode())
            if header.get("format") != "window-cnn/1" or header.get("num_params") != num_params():
                raise ValueError("%s is not a window-network checkpoint of this layout" % path)
            net = cls(params=z["params"], device=device)
            net.m.copy_(torch.from_numpy(z["m"]))
            net.v.copy_(torch.from_numpy(z["v"]))
        net.step = int(header["step"])
        net.header = header
        return net


def prepare_input(coarse_disp, coarse_left, W, H, n, x0=None, stream=None):
    if x0 is None:
        x0 = torch.empty((n, H, W, CH), dtype=torch.int16, device=coarse_disp.device)
    S._check(_lib.sgm_cnn_prepare_input(_c(coarse_disp), _c(coarse_left), W, H, n, _c(x0),
                                        S._stream(stream)), "sgm_cnn_prepare_input")
    return x0


def label_downsample4(label, out=None, stream=None):
    H, W = label.shape
    if out is None:
        out = torch.empty((H // 4, W // 4), dtype=torch.float32, device=label.device)
    S._check(_lib.sgm_label_downsample4(_c(label), W, H, _c(out), S._stream(stream)),
             "sgm_label_downsample4")
    return out


ALWAYS_FALL_BACK = -2 ** 31  # fallback margin: every low-confidence pixel falls back


def window_map(coarse_disp, out, W, H, ndisp, w, tau, lo=None, mask=None, row_stats=None,
               nfallback=None, fallback_margin=0, stream=None):
    Hc, Wc = coarse_disp.shape[-2:]
    if lo is None:
        lo = torch.empty((H, W), dtype=torch.int32, device=coarse_disp.device)
    S._check(_lib.sgm_window_map(_c(coarse_disp), _c(out), Wc, Hc, W, H, ndisp, w, float(tau), int(fallback_margin),
                                 _c(lo), _c(mask), _c(row_stats), _c(nfallback), S._stream(stream)),
             "sgm_window_map")
    return lo


def window_map_batch(coarse_disp, out, W, H, ndisp, w, tau, lo, mask, row_stats, nfallback, fallback_margin=0,
                     stream=None):
    """window_map for a stack of n images (every buffer packed per image)."""
    n, Hc, Wc = coarse_disp.shape
    S._check(_lib.sgm_window_map_batch(_c(coarse_disp), _c(out), Wc, Hc, W, H, ndisp, w, float(tau),
                                       int(fallback_margin), n, _c(lo), _c(mask), _c(row_stats), _c(nfallback),
                                       S._stream(stream)), "sgm_window_map_batch")
    return lo


def fallback_merge(mask, band_int, band_sub, y0, x0, disp_int, disp_sub, stream=None):
    H, W = disp_int.shape
    rows, cols = band_int.shape
    S._check(_lib.sgm_fallback_merge(_c(mask), _c(band_int), _c(band_sub), W, H, int(y0), int(rows), int(x0),
                                     int(cols), _c(disp_int), _c(disp_sub), S._stream(stream)),
             "sgm_fallback_merge")


def fallback_merge_rects(mask, table, nrects, max_rows, max_cols, band_int, band_sub, disp_int, disp_sub,
                         stream=None):
    """Every rectangle of a batch in one launch: `table` int32 device
    [>= nrects, 6] rows (frame, y0, rows, x0, cols, band offset); mask,
    disp_int, disp_sub [n, H, W]; band_int / band_sub flat."""
    n, H, W = disp_int.shape
    S._check(_lib.sgm_fallback_merge_rects(_c(mask), _c(table), int(nrects), int(max_rows), int(max_cols), W, H, n,
                                           _c(band_int), _c(band_sub), int(band_int.numel()), _c(disp_int),
                                           _c(disp_sub), S._stream(stream)), "sgm_fallback_merge_rects")


def fallback_rects(row_stats, W, ndisp, r, margin=32, full_fraction=0.5):
    """Rectangles [(y0, y1, x0, x1)] for the full-range fallback from the
    per-row statistics of the window map (int32 [3, H]: fallback count,
    leftmost and rightmost fallback column).  Each row with fallback pixels
    is widened by `margin` rows both ways; overlapping or touching rows form
    one band, whose columns span its fallback pixels widened by margin + r
    on the right and margin + ndisp - 1 + r on the left (every disparity of
    the widened region then reads its right-image pixel, and the census
    neighbours, inside the rectangle).  Past `full_fraction` of the frame's
    area the whole frame is one rectangle."""
    stats = np.asarray(row_stats)
    count, xmin, xmax = stats[0], stats[1], stats[2]
    H = count.shape[0]
    flagged = np.flatnonzero(count > 0)
    if flagged.size == 0:
        return []
    lo = np.maximum(flagged - margin, 0)
    hi = np.minimum(flagged + margin + 1, H)
    # a new band starts where the widened row does not reach the previous ones
    starts = np.ones(flagged.size, bool)
    starts[1:] = lo[1:] > np.maximum.accumulate(hi)[:-1]
    idx = np.flatnonzero(starts)
    ends = np.r_[idx[1:], flagged.size]
    rects = []
    for a, b in zip(idx, ends):
        rows = flagged[a:b]
        xl, xr = int(xmin[rows].min()), int(xmax[rows].max())
        rects.append((int(lo[a]), int(hi[a:b].max()), max(0, xl - margin - (ndisp - 1) - r),
                      min(W, xr + margin + r + 1)))
    if sum((y1 - y0) * (x1 - x0) for y0, y1, x0, x1 in rects) > full_fraction * H * W:
        return [(0, H, 0, W)]
    return rects


class LearnedWindowMatcher:
    """Coarse full-range SGM -> window network -> per-pixel-window SGM ->
    full-range fallback, for batches of `batch` pairs of one size."""

    def __init__(self, width, height, batch=1, ndisp=192, window=16, census=7, npaths=8, p1=10,
                 p2=120, net=None, tau=0.5, margin=32, full_fraction=0.5, fallback_streams=3, autotune=True,
                 fallback_margin=8, device="cuda"):
        if width % 4 or height % 4 or ndisp % 4:
            raise ValueError("width, height and ndisp must be multiples of 4")
        self.W, self.H, self.D, self.w, self.n = width, height, ndisp, window, batch
        self.Wc, self.Hc = width // 4, height // 4
        self.census, self.npaths, self.p1, self.p2 = census, npaths, p1, p2
        self.tau, self.margin, self.full_fraction = tau, margin, full_fraction
        # low-confidence pixels fall back only while x - 4 coarse >= this:
        # by default, unless the coarse match lies within two coarse pixels
        # of the left image edge, where the scene point is taken as outside
        # the right camera's view (ALWAYS_FALL_BACK: every one of them)
        self.fallback_margin = int(fallback_margin)
        self.device = dev = torch.device(device)
        self.net = net if net is not None else WindowNet.load(DEFAULT_WEIGHTS, device=device)
        n, Hc, Wc = batch, self.Hc, self.Wc
        self.cl = torch.empty((n, Hc, Wc), dtype=torch.uint8, device=dev)
        self.cr = torch.empty_like(self.cl)
        self.cdi = torch.empty((n, Hc, Wc), dtype=torch.int16, device=dev)
        self.cds = torch.empty((n, Hc, Wc), dtype=torch.float32, device=dev)
        self.coarse = S.Batch([dict(left=self.cl[i], right=self.cr[i], ndisp=ndisp // 4, disp_int=self.cdi[i],
                                    disp_sub=self.cds[i]) for i in range(n)],
                              census=census, npaths=npaths, p1=p1, p2=p2, device=dev)
        if autotune:
            # launch shape of the quarter-scale batch (timed once on these buffers)
            self.cl.zero_()
            self.cr.zero_()
            self.coarse.autotune()
        self.x0 = torch.empty((n, Hc, Wc, CH), dtype=torch.int16, device=dev)
        self.out = torch.empty((n, Hc, Wc, OUT_CH), dtype=torch.float32, device=dev)
        fine_plan = S.sgm_plan(width, height, census, window, npaths, p1, p2)
        try:
            nb = ctypes.c_size_t()
            S._check(_lib.sgm_workspace_size_win_batch(fine_plan, n, ctypes.byref(nb)), "sgm_workspace_size_win_batch")
            fine_ws = int(nb.value)
        finally:
            S.sgm_plan_free(fine_plan)
        self.fine_ws = torch.empty(fine_ws, dtype=torch.uint8, device=dev)  # every pair's slice
        self.fine = S.Matcher(width, height, census=census, ndisp=window, npaths=npaths, p1=p1, p2=p2,
                              device=dev, workspace=self.fine_ws)
        self.lo = torch.empty((n, height, width), dtype=torch.int32, device=dev)
        self.mask = torch.empty((n, height, width), dtype=torch.uint8, device=dev)
        self.stats = torch.zeros((n, 3, height), dtype=torch.int32, device=dev)
        self.stats_host = torch.zeros((n, 3, height), dtype=torch.int32, pin_memory=True)
        self.nfallback = torch.zeros((n,), dtype=torch.int32, device=dev)
        self.dint = torch.empty((n, height, width), dtype=torch.int16, device=dev)
        self.dsub = torch.empty((n, height, width), dtype=torch.float32, device=dev)
        # full-range fallback: plain SGM of each rectangle on a side stream,
        # which starts as soon as the window maps are done and runs beside
        # the windowed SGM; one full-frame workspace, plans per rectangle
        # size (host objects), results in an arena merged on the main stream
        full = S.sgm_plan(width, height, census, ndisp, npaths, p1, p2)
        try:
            need = S.sgm_workspace_size(full)
        finally:
            S.sgm_plan_free(full)
        # pair i's rectangles go to side stream i % len(streams), each stream
        # with its own workspace, so the small launches also overlap each other.
        # Streams share the process's hardware queues (four by default, given
        # out in turn as streams are made): a fallback stream that lands on
        # the queue of the stream running the windowed SGM waits behind it.
        # Measured on a batch of 16 x 1920x1080 (stream made after this
        # object): 3 side streams 4.22 ms per batch with the fallback done
        # 0.03 ms after the windowed SGM, 4 streams 4.51 ms (0.41 ms after),
        # 2 streams 4.39 ms, 1 stream 4.57 ms.
        nst = max(1, min(fallback_streams, n))
        self.fb_streams = [torch.cuda.Stream(device=dev) for _ in range(nst)]
        self.fb_ws = [torch.empty(need, dtype=torch.uint8, device=dev) for _ in range(nst)]
        self.fb_int = torch.empty(n * height * width, dtype=torch.int16, device=dev)
        self.fb_sub = torch.empty(n * height * width, dtype=torch.float32, device=dev)
        self.ev_maps = torch.cuda.Event()
        self.ev_fb = [torch.cuda.Event() for _ in range(nst)]
        # the batch's rectangle table for the one-launch merge (pinned host
        # copy uploaded on the main stream)
        self.max_rects = 4096
        self.rect_host = torch.zeros((self.max_rects, 6), dtype=torch.int32, pin_memory=True)
        self.rect_dev = torch.zeros((self.max_rects, 6), dtype=torch.int32, device=dev)
        self._full = [{} for _ in range(nst)]
        self.last_rects = []

    def _full_matcher(self, j, rows, cols):
        cache = self._full[j]
        key = (rows, cols)
        m = cache.pop(key, None)
        if m is None:
            m = S.Matcher(cols, rows, census=self.census, ndisp=self.D, npaths=self.npaths, p1=self.p1,
                          p2=self.p2, device=self.device, workspace=self.fb_ws[j])
            while len(cache) >= 256:  # plans are host objects; keep the most recent
                cache.pop(next(iter(cache)))
        cache[key] = m
        return m

    STAGES = ("reduce", "coarse_sgm", "network", "window_map", "windowed_sgm", "fallback_merge")

    def windows(self, left, right, stream=None, events=None):
        """Steps 1-5 for left, right uint8 [n, H, W]: fills lo, mask, stats,
        nfallback, dint and dsub (records ev_maps once the maps are done).
        `events` (optional, 7 timing events) are recorded on the stream
        before the first stage and after each of STAGES."""
        n = self.n
        if tuple(left.shape) != (n, self.H, self.W) or tuple(right.shape) != (n, self.H, self.W):
            raise ValueError("left and right must be uint8 [%d, %d, %d]" % (n, self.H, self.W))
        main = stream if stream is not None else torch.cuda.current_stream(self.device)

        def mark(k):
            if events is not None:
                events[k].record(main)

        mark(0)
        S.sgm_downsample4_batch(left, self.cl, main)
        S.sgm_downsample4_batch(right, self.cr, main)
        mark(1)
        self.coarse.run(main)
        mark(2)
        prepare_input(self.cds, self.cl, self.Wc, self.Hc, n, self.x0, main)
        self.net.infer(self.x0, self.out, self.Wc, self.Hc, n, main)
        mark(3)
        window_map_batch(self.cds, self.out, self.W, self.H, self.D, self.w, self.tau, self.lo, self.mask,
                         self.stats, self.nfallback, self.fallback_margin, main)
        mark(4)
        self.ev_maps.record(main)
        if self.w == 16:
            self.fine.match_win_batch(left, right, self.lo, disp_int=self.dint, disp_sub=self.dsub,
                                      workspace=self.fine_ws, stream=main)
        else:
            for i in range(n):
                self.fine.match_win(left[i], right[i], self.lo[i], disp_int=self.dint[i], disp_sub=self.dsub[i],
                                    stream=main)
        mark(5)

    def fallback(self, left, right, stream=None, events=None):
        """Step 6: waits on the host for the window maps only; the
        rectangles' plain SGM runs on the side stream beside the windowed
        SGM, and the merge follows both on the main stream."""
        main = stream if stream is not None else torch.cuda.current_stream(self.device)
        fb0 = self.fb_streams[0]
        for st in self.fb_streams:
            st.wait_event(self.ev_maps)
        with torch.cuda.stream(fb0):
            self.stats_host.copy_(self.stats, non_blocking=True)
        fb0.synchronize()
        stats = self.stats_host.numpy()
        self.last_rects = []
        merges = []
        used = 0
        for i in range(self.n):
            rects = fallback_rects(stats[i], self.W, self.D, self.census // 2, self.margin, self.full_fraction)
            self.last_rects.append(rects)
            j = i % len(self.fb_streams)
            for y0, y1, x0, x1 in rects:
                h, w = y1 - y0, x1 - x0
                bi = self.fb_int[used:used + h * w].view(h, w)
                bs = self.fb_sub[used:used + h * w].view(h, w)
                used += h * w
                self._full_matcher(j, h, w).match_at(left[i], right[i], y0, x0, disp_int=bi, disp_sub=bs,
                                                     stream=self.fb_streams[j])
                merges.append((i, y0, x0, bi, bs))
        if merges:
            for st, ev in zip(self.fb_streams, self.ev_fb):
                ev.record(st)
                main.wait_event(ev)
            if len(merges) <= self.max_rects:
                # one launch for every rectangle (bands of a frame never overlap)
                tab = self.rect_host.numpy()
                off = 0
                for k, (i, y0, x0, bi, bs) in enumerate(merges):
                    h, w = bi.shape
                    tab[k] = (i, y0, h, x0, w, off)
                    off += h * w
                with torch.cuda.stream(main):
                    self.rect_dev[:len(merges)].copy_(self.rect_host[:len(merges)], non_blocking=True)
                fallback_merge_rects(self.mask, self.rect_dev, len(merges), max(b.shape[0] for _, _, _, b, _ in merges),
                                     max(b.shape[1] for _, _, _, b, _ in merges), self.fb_int[:off],
                                     self.fb_sub[:off], self.dint, self.dsub, main)
            else:
                for i, y0, x0, bi, bs in merges:
                    fallback_merge(self.mask[i], bi, bs, y0, x0, self.dint[i], self.dsub[i], main)
        if events is not None:
            events[6].record(main)

    def match(self, left, right, stream=None, events=None):
        """Returns (disp_int int16 [n,H,W], disp_sub float32 [n,H,W]) device
        tensors.  `events`: optional 7 timing events for the stages (STAGES)."""
        self.windows(left, right, stream, events)
        self.fallback(left, right, stream, events)
        return self.dint, self.dsub
