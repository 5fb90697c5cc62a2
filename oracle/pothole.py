"""CPU oracle of the pothole threshold and labelling (test infrastructure
only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It shares no code with the HIP path.

Sec. II-E detects potholes on the transformed disparity map D2 (eq. (13)).
The superpixel step (SLIC, D3) is not part of this oracle: the threshold is
applied to D2 pixel by pixel.

Vectors: each pixel p whose 3x3 neighbourhood lies inside the image, with p
and its 8 neighbours selected (mask non-zero, or no mask) and finite, gives
g = [D2(p), sum of D2 over the 8 neighbours] (the neighbour sum taken in
float64 in row-major neighbour order).

Threshold search (eq. (14), (15)): candidates t_r = lo + k b, b = (hi - lo) /
nbins, k = 1 .. nbins - 1.  For a candidate, region 1 (foreground) holds the
vectors with both components below the diagonal split (g0 < t_r and
g1 < 8 t_r), region 2 (background) those with both at or above it; the mixed
regions 3 and 4 are left out.  E2(t_r) = sum over regions 1 and 2 of
|g|^2 - n1 |mu1|^2 - n2 |mu2|^2 (eq. (15)); t_r minimises E2 over the
candidates whose two regions are both non-empty (the smallest k on a tie).
The comparisons go through bin indices computed in float64,
i = clamp(floor((g0 - lo) / b), 0, nbins - 1) and
j = clamp(floor((g1 - 8 lo) / (8 b)), 0, nbins - 1): g is in region 1 for
index k when max(i, j) < k and in region 2 when min(i, j) >= k.
Then t_s = t_r - delta_PD (eq. (14)).

Labelling: pothole pixels are selected, finite pixels with D2 < t_s;
connected components with 8-connectivity; each component is labelled
1 + the smallest row-major index among its pixels, other pixels 0.
"""
from __future__ import annotations

import collections
import math

import numpy as np

OFFSETS = [(dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dy, dx) != (0, 0)]


def vectors(d2, mask=None):
    """(g0, g1, valid) as float64 / bool arrays [H][W]."""
    D = np.asarray(d2, dtype=np.float32).astype(np.float64)
    H, W = D.shape
    sel = np.isfinite(D)
    if mask is not None:
        sel &= np.asarray(mask) != 0
    valid = np.zeros((H, W), bool)
    g1 = np.zeros((H, W), np.float64)
    if H >= 3 and W >= 3:
        ok = sel[1:-1, 1:-1].copy()
        acc = np.zeros((H - 2, W - 2), np.float64)
        for dy, dx in OFFSETS:
            nb = D[1 + dy:H - 1 + dy, 1 + dx:W - 1 + dx]
            ok &= sel[1 + dy:H - 1 + dy, 1 + dx:W - 1 + dx]
            acc = acc + np.where(np.isfinite(nb), nb, 0.0)
        valid[1:-1, 1:-1] = ok
        g1[1:-1, 1:-1] = acc
    return D, g1, valid


def bins(g0, g1, lo, hi, nbins):
    b = (hi - lo) / nbins
    i = np.clip(np.floor((g0 - lo) / b), 0, nbins - 1).astype(np.int64)
    j = np.clip(np.floor((g1 - 8.0 * lo) / (8.0 * b)), 0, nbins - 1).astype(np.int64)
    return i, j


def e2_curve(d2, lo, hi, nbins, mask=None):
    """E2 (eq. (15)), n1 and n2 for k = 0 .. nbins (entries 0 and nbins
    unused: NaN / 0)."""
    g0, g1, valid = vectors(d2, mask)
    g0, g1 = g0[valid], g1[valid]
    i, j = bins(g0, g1, lo, hi, nbins)
    hi_idx, lo_idx = np.maximum(i, j), np.minimum(i, j)
    sq = g0 * g0 + g1 * g1
    E2 = np.full(nbins + 1, np.nan)
    n1 = np.zeros(nbins + 1, np.int64)
    n2 = np.zeros(nbins + 1, np.int64)
    for k in range(1, nbins):
        r1, r2 = hi_idx < k, lo_idx >= k
        n1[k], n2[k] = int(r1.sum()), int(r2.sum())
        e = 0.0
        for r, n in ((r1, n1[k]), (r2, n2[k])):
            if n:
                s0, s1 = g0[r].sum(), g1[r].sum()
                e += sq[r].sum() - (s0 * s0 + s1 * s1) / n
        E2[k] = e
    return E2, n1, n2


def threshold(d2, lo, hi, nbins, delta_pd, mask=None):
    """dict(status, k, t_r, t_s, e2, n1, n2); status 1 when no candidate has
    two non-empty regions."""
    E2, n1, n2 = e2_curve(d2, lo, hi, nbins, mask)
    best = None
    for k in range(1, nbins):
        if n1[k] > 0 and n2[k] > 0 and (best is None or E2[k] < E2[best]):
            best = k
    if best is None:
        return dict(status=1, k=0, t_r=math.nan, t_s=math.nan, e2=math.nan, n1=0, n2=0)
    t_r = lo + best * ((hi - lo) / nbins)
    return dict(status=0, k=best, t_r=t_r, t_s=t_r - delta_pd, e2=float(E2[best]), n1=int(n1[best]),
                n2=int(n2[best]))


def label(d2, t_s, mask=None):
    """Pothole labels int32 [H][W] (8-connected components of D2 < t_s)."""
    D = np.asarray(d2, dtype=np.float32)
    H, W = D.shape
    fg = np.isfinite(D) & (D.astype(np.float64) < t_s)
    if mask is not None:
        fg &= np.asarray(mask) != 0
    lab = np.zeros((H, W), np.int32)
    seen = np.zeros((H, W), bool)
    for y0, x0 in zip(*np.nonzero(fg)):  # row-major: a component is first met at its smallest index
        if seen[y0, x0]:
            continue
        name = int(y0) * W + int(x0) + 1
        seen[y0, x0] = True
        queue = collections.deque([(y0, x0)])
        while queue:
            y, x = queue.popleft()
            lab[y, x] = name
            for dy, dx in OFFSETS:
                yy, xx = y + dy, x + dx
                if 0 <= yy < H and 0 <= xx < W and fg[yy, xx] and not seen[yy, xx]:
                    seen[yy, xx] = True
                    queue.append((yy, xx))
    return lab


def prune_single_superpixel(labels, superpixels):
    """Sec. III-B counts a detected pothole made of a single superpixel as a
    false one: every component of `labels` (0 = none) whose pixels all lie
    in one superpixel of `superpixels` is removed (set to 0); the others
    keep their labels."""
    lab = np.array(labels, dtype=np.int32, copy=True)
    sp = np.asarray(superpixels)
    for name in np.unique(lab[lab > 0]):
        if np.unique(sp[lab == name]).size == 1:
            lab[lab == name] = 0
    return lab

