"""CPU oracle of the search-window CNN (test infrastructure only).

A 4-layer 3x3 convolutional network, 16 channels everywhere (the input's
unused channels are zero), zero padding, ReLU after the first three
layers.  Output channel 0 is the window-centre offset (coarse pixels),
channel 1 the confidence logit.  Plain numpy in float64; where the GPU
rounds to bfloat16 (weights, activations, gradients fed to the matrix
units) this oracle rounds the same operands (round to nearest even), so the
two differ only by the order of float32 accumulation.

Parameter vector (float32): for each layer l = 0..3, W[l] as [tap][co][ci]
with tap = (dy + 1) * 3 + (dx + 1), then b[l] as [co].
"""
from __future__ import annotations

import numpy as np

CH = 16
LAYERS = 4
PER_LAYER = 9 * CH * CH + CH
NPARAMS = LAYERS * PER_LAYER
TAPS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16(x):
    """Round to the nearest bfloat16 (ties to even); returned as float64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    Ws, bs = [], []
    for l in range(LAYERS):
        base = l * PER_LAYER
        Ws.append(p[base:base + 9 * CH * CH].reshape(9, CH, CH))
        bs.append(p[base + 9 * CH * CH: base + PER_LAYER])
    return Ws, bs


def conv3x3(x, W, b):
    """out[n,y,x,co] = b[co] + sum_t sum_ci W[t,co,ci] x[n,y+dy,x+dx,ci]."""
    n, H, Wd, _ = x.shape
    xp = np.zeros((n, H + 2, Wd + 2, CH))
    xp[:, 1:-1, 1:-1] = x
    out = np.broadcast_to(b, (n, H, Wd, CH)).copy()
    for t, (dy, dx) in enumerate(TAPS):
        patch = xp[:, 1 + dy: 1 + dy + H, 1 + dx: 1 + dx + Wd]
        out += patch @ W[t].T
    return out


def forward(params, x0, rounding=True):
    """Returns (hidden activations X1..X3, final output).  Hidden
    activations are bfloat16 values; the output is float."""
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    Ws, bs = unpack(params)
    x = rnd(x0)
    acts = []
    for l in range(LAYERS):
        y = conv3x3(x, rnd(Ws[l]), bs[l])
        if l < LAYERS - 1:
            x = rnd(np.maximum(y, 0.0))
            acts.append(x)
        else:
            out = y
    return acts, out


def loss_and_grad(out, coarse, label_c):
    """Huber loss on the centre offset (target label - coarse, coarse px)
    plus a logistic loss on the confidence (target: |offset error| < 1);
    mean over pixels.  Returns (loss, d loss / d out)."""
    out = np.asarray(out, dtype=np.float64)
    N = out.shape[0] * out.shape[1] * out.shape[2]
    off, logit = out[..., 0], out[..., 1]
    e = off - (np.asarray(label_c, np.float64) - np.asarray(coarse, np.float64))
    ae = np.abs(e)
    huber = np.where(ae <= 1.0, 0.5 * e * e, ae - 0.5)
    c = (ae < 1.0).astype(np.float64)
    bce = np.maximum(logit, 0.0) - c * logit + np.log1p(np.exp(-np.abs(logit)))
    loss = (huber.sum() + bce.sum()) / N
    g = np.zeros_like(out)
    g[..., 0] = np.clip(e, -1.0, 1.0) / N
    g[..., 1] = (1.0 / (1.0 + np.exp(-logit)) - c) / N
    return loss, g


def conv3x3_backward(x, W, dy):
    """Gradients of conv3x3 w.r.t. x, W and b for upstream dy."""
    n, H, Wd, _ = x.shape
    xp = np.zeros((n, H + 2, Wd + 2, CH))
    xp[:, 1:-1, 1:-1] = x
    dW = np.zeros((9, CH, CH))
    dxp = np.zeros_like(xp)
    for t, (ddy, ddx) in enumerate(TAPS):
        patch = xp[:, 1 + ddy: 1 + ddy + H, 1 + ddx: 1 + ddx + Wd]
        dW[t] = np.einsum("nyxo,nyxi->oi", dy, patch)
        dxp[:, 1 + ddy: 1 + ddy + H, 1 + ddx: 1 + ddx + Wd] += dy @ W[t]
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1], dW, db


def backward(params, x0, acts, dout, rounding=True):
    """Parameter gradient (flat, float64) of the loss whose output gradient
    is dout, through the four layers."""
    rnd = bf16 if rounding else (lambda a: np.asarray(a, dtype=np.float64))
    Ws, _ = unpack(params)
    inputs = [rnd(x0)] + list(acts)
    grads = [None] * LAYERS
    dy = rnd(dout)
    for l in range(LAYERS - 1, -1, -1):
        dx, dW, db = conv3x3_backward(inputs[l], rnd(Ws[l]), dy)
        grads[l] = np.concatenate([dW.ravel(), db])
        if l > 0:
            dy = rnd(dx * (inputs[l] > 0))
    return np.concatenate(grads)


def adam(params, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), float64 reference."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def prepare_input(coarse_disp, coarse_left):
    """Network input: channel 0 = coarse disparity / 16, channel 1 =
    intensity / 255 - 1/2, channel 2 = min(column - coarse disparity, 16) / 16
    (how far the coarse match lies from the left image border, saturated),
    channels 3..15 zero.  Float32 arithmetic, as the input is built."""
    H, W = coarse_disp.shape
    cd = np.asarray(coarse_disp, np.float32)
    col = np.broadcast_to(np.arange(W, dtype=np.float32)[None, :], (H, W))
    x = np.zeros((1, H, W, CH))
    x[0, :, :, 0] = cd / np.float32(16.0)
    x[0, :, :, 1] = np.asarray(coarse_left, np.float32) / np.float32(255.0) - np.float32(0.5)
    x[0, :, :, 2] = np.minimum(col - cd, np.float32(16.0)) / np.float32(16.0)
    return x


def confidence_threshold(tau):
    """Logit threshold of the confidence probability tau: a pixel is
    confident when sigmoid(logit) > tau, i.e. logit > log(tau / (1 - tau));
    tau <= 0 accepts every logit, tau >= 1 none."""
    if tau <= 0.0:
        return np.float32(-np.inf)
    if tau >= 1.0:
        return np.float32(np.inf)
    return np.float32(np.log(tau / (1.0 - tau)))


def window_map(coarse_disp, out, W, H, D, w, tau, fallback_margin=None):
    """Per-pixel window start and fallback mask.  Each full-resolution pixel
    takes its coarse pixel (x // 4, y // 4, clamped to the coarse grid).
    Confident pixels centre the window on 4 * (coarse + offset), the others
    on 4 * coarse; lo = clamp(floor(centre + 1/2) - w/2, 0, D - w).  A
    pixel that is not confident is marked for the full-range fallback when
    fallback_margin is None, or else when its coarse match x - 4 * coarse
    (float32) is at least fallback_margin.
    Returns (lo int32 [H, W], number of fallback pixels, mask uint8 [H, W])."""
    Hc, Wc = coarse_disp.shape
    ys = np.minimum(np.arange(H) // 4, Hc - 1)
    xs = np.minimum(np.arange(W) // 4, Wc - 1)
    cd = np.asarray(coarse_disp, np.float32)[ys][:, xs]
    off = np.asarray(out[0, :, :, 0], np.float32)[ys][:, xs]
    lg = np.asarray(out[0, :, :, 1], np.float32)[ys][:, xs]
    conf = lg > confidence_threshold(tau)
    centre_c = np.where(conf, cd + off, cd).astype(np.float32)
    centre = np.float32(4.0) * centre_c
    lo = np.floor(centre + np.float32(0.5)).astype(np.int64) - w // 2
    fb = ~conf
    if fallback_margin is not None:
        match = np.arange(W, dtype=np.float32)[None, :] - centre  # x - 4 coarse where not confident
        fb &= match >= np.float32(fallback_margin)
    mask = fb.astype(np.uint8)
    return np.clip(lo, 0, D - w).astype(np.int32), int(mask.sum()), mask


def fallback_rects(mask, margin, full_fraction, ndisp, r):
    """Rectangles (y0, y1, x0, x1) for the full-range fallback.  Rows that
    hold a fallback pixel, widened by `margin` rows both ways, form bands
    (overlapping or touching ones joined).  A band spans the columns of its
    fallback pixels, widened by margin + r on the right and by
    margin + (ndisp - 1) + r on the left, so that every disparity of the
    widened region finds its right-image pixel (and census neighbours)
    inside the rectangle.  When the rectangles would cover more than
    `full_fraction` of the frame, the whole frame is one rectangle."""
    H, W = mask.shape
    rows = [y for y in range(H) if mask[y].any()]
    bands = []  # [y0, y1, xmin, xmax]
    for y in rows:
        cols = [x for x in range(W) if mask[y, x]]
        a, b = max(0, y - margin), min(H, y + margin + 1)
        if bands and a <= bands[-1][1]:
            bands[-1][1] = max(bands[-1][1], b)
            bands[-1][2] = min(bands[-1][2], cols[0])
            bands[-1][3] = max(bands[-1][3], cols[-1])
        else:
            bands.append([a, b, cols[0], cols[-1]])
    rects = [(a, b, max(0, xl - margin - (ndisp - 1) - r), min(W, xr + margin + r + 1))
             for a, b, xl, xr in bands]
    if sum((b - a) * (x1 - x0) for a, b, x0, x1 in rects) > full_fraction * H * W:
        return [(0, H, 0, W)]
    return rects


def merge_fallback(win_int, win_sub, mask, rects, results):
    """Final disparities: the windowed result, replaced on fallback pixels by
    the full-range result of the rectangle that holds them."""
    dint = np.array(win_int, copy=True)
    dsub = np.array(win_sub, copy=True)
    for (y0, y1, x0, x1), (bi, bs) in zip(rects, results):
        m = mask[y0:y1, x0:x1].astype(bool)
        dint[y0:y1, x0:x1][m] = bi[m]
        dsub[y0:y1, x0:x1][m] = bs[m]
    return dint, dsub
