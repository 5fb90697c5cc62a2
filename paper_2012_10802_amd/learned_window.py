"""Learned search windows (the learned-window form of the SGM path).

Pipeline per pair, every step a HIP kernel behind the C ABI:
  1. 4 x 4 box reduction of both images (quarter resolution);
  2. plain full-range SGM on the quarter-resolution pair (ndisp / 4
     disparities): the coarse disparity;
  3. the window network (four 3x3 convolutions, 16 channels, bfloat16 on the
     matrix cores) on [coarse disparity, coarse left image]: a centre offset
     and a confidence logit per coarse pixel;
  4. the window map: per full-resolution pixel a 16-wide window centred on
     4 * (coarse + offset) where the network is confident, on 4 * coarse
     (the full-range estimate) where it is not;
  5. SGM over the per-pixel windows at full resolution.

Training: pairs from the road generator, labelled by full-range plain SGM at
full resolution on the GPU; Adam on float32 master weights with the
hand-written forward, loss, backward and optimiser kernels.  Checkpoints
are plain arrays (numpy .npz, no pickles) with a JSON header.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np
import torch

from . import sgm as S

CH = 16
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "window_cnn.npz")
_lib = S.library()


def _c(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def num_params() -> int:
    return int(_lib.sgm_cnn_num_params())


def init_params(seed=0):
    """He-normal weights for the used input channels, zero biases; the last
    layer starts small."""
    rng = np.random.default_rng(seed)
    per = 9 * CH * CH + CH
    p = np.zeros(4 * per, np.float32)
    for l in range(4):
        fan_in = 9 * (2 if l == 0 else CH)
        Wl = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(9, CH, CH)).astype(np.float32)
        if l == 0:
            Wl[:, :, 2:] = 0.0
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
        self.wf = torch.empty(4 * 9 * CH * CH, dtype=torch.int16, device=self.device)
        self.wb = torch.empty_like(self.wf)
        S._check(_lib.sgm_cnn_pack_weights(_c(self.params), _c(self.wf), _c(self.wb), S._stream()),
                 "sgm_cnn_pack_weights")

    # --- buffers for n images of W x H
    def buffers(self, W, H, n):
        act = torch.empty((3, n, H, W, CH), dtype=torch.int16, device=self.device)
        out = torch.empty((n, H, W, CH), dtype=torch.float32, device=self.device)
        return act, out

    def forward(self, x0, acts, out, W, H, n, stream=None):
        S._check(_lib.sgm_cnn_forward(_c(self.wf), _c(self.params), _c(x0), W, H, n, _c(acts), _c(out),
                                      S._stream(stream)), "sgm_cnn_forward")
        return out

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

    def train_buffers(self, W, H, n):
        acts, out = self.buffers(W, H, n)
        dy = torch.empty((n, H, W, CH), dtype=torch.int16, device=self.device)
        scratch = torch.empty(int(_lib.sgm_cnn_scratch_bytes(W, H, n)), dtype=torch.uint8,
                              device=self.device)
        loss = torch.zeros(2, dtype=torch.float32, device=self.device)
        return acts, out, dy, scratch, loss

    # --- checkpoints: plain arrays + JSON header (no pickles)
    def save(self, path, extra=None):
        header = {"format": "window-cnn/1", "step": self.step, "num_params": num_params()}
        header.update(extra or {})
        np.savez(path, params=self.params.cpu().numpy(), m=self.m.cpu().numpy(),
                 v=self.v.cpu().numpy(),
                 header=np.frombuffer(json.dumps(header).encode(), dtype=np.uint8))

    @classmethod
    def load(cls, path, device="cuda"):
        with np.load(path, allow_pickle=False) as z:
            header = json.loads(bytes(z["header"]).decode())
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


def window_map(coarse_disp, out, W, H, ndisp, w, threshold, lo=None, nfallback=None, stream=None):
    Hc, Wc = coarse_disp.shape[-2:]
    if lo is None:
        lo = torch.empty((H, W), dtype=torch.int32, device=coarse_disp.device)
    S._check(_lib.sgm_window_map(_c(coarse_disp), _c(out), Wc, Hc, W, H, ndisp, w, float(threshold),
                                 _c(lo), _c(nfallback), S._stream(stream)), "sgm_window_map")
    return lo


class LearnedWindowMatcher:
    """Coarse full-range SGM -> window network -> per-pixel-window SGM."""

    def __init__(self, width, height, ndisp=192, window=16, census=7, npaths=8, p1=10, p2=120,
                 net=None, threshold=0.0, device="cuda"):
        if width % 4 or height % 4 or ndisp % 4:
            raise ValueError("width, height and ndisp must be multiples of 4")
        self.W, self.H, self.D, self.w = width, height, ndisp, window
        self.Wc, self.Hc = width // 4, height // 4
        self.threshold = threshold
        self.device = torch.device(device)
        self.net = net if net is not None else WindowNet.load(DEFAULT_WEIGHTS, device=device)
        self.coarse = S.Matcher(self.Wc, self.Hc, census=census, ndisp=ndisp // 4, npaths=npaths,
                                p1=p1, p2=p2, device=device)
        self.fine = S.Matcher(width, height, census=census, ndisp=window, npaths=npaths, p1=p1, p2=p2,
                              device=device)
        dev = self.device
        self.cl = torch.empty((self.Hc, self.Wc), dtype=torch.uint8, device=dev)
        self.cr = torch.empty_like(self.cl)
        self.cdi = torch.empty((self.Hc, self.Wc), dtype=torch.int16, device=dev)
        self.cds = torch.empty((self.Hc, self.Wc), dtype=torch.float32, device=dev)
        self.x0 = torch.empty((1, self.Hc, self.Wc, CH), dtype=torch.int16, device=dev)
        self.acts, self.out = self.net.buffers(self.Wc, self.Hc, 1)
        self.lo = torch.empty((height, width), dtype=torch.int32, device=dev)
        self.nfallback = torch.zeros(1, dtype=torch.int32, device=dev)
        self.dint = torch.empty((height, width), dtype=torch.int16, device=dev)
        self.dsub = torch.empty((height, width), dtype=torch.float32, device=dev)

    def match(self, left, right, stream=None):
        """Returns (disp_int, disp_sub, lo, nfallback) device tensors."""
        S.sgm_downsample4(left, self.cl, stream)
        S.sgm_downsample4(right, self.cr, stream)
        self.coarse.match(self.cl, self.cr, disp_int=self.cdi, disp_sub=self.cds, stream=stream)
        prepare_input(self.cds, self.cl, self.Wc, self.Hc, 1, self.x0, stream)
        self.net.forward(self.x0, self.acts, self.out, self.Wc, self.Hc, 1, stream)
        self.nfallback.zero_()
        window_map(self.cds, self.out, self.W, self.H, self.D, self.w, self.threshold, self.lo,
                   self.nfallback, stream)
        self.fine.match_win(left, right, self.lo, disp_int=self.dint, disp_sub=self.dsub, stream=stream)
        return self.dint, self.dsub, self.lo, self.nfallback
