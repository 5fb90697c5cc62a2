"""CPU oracle of the superpixel step on the transformed disparity map
(test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It shares no code with the HIP path.

Sec. II-D groups D2 into superpixels with SLIC and Sec. II-E replaces each
superpixel by the mean of its transformed disparities (D3).  SLIC, as the
paper summarises it: cluster centres on a regular grid, each moved to the
lowest-gradient position of its 3x3 neighbourhood, then k-means iterations
in which every pixel joins the nearest centre among those whose search
range covers it, and every centre moves to the mean of its pixels.
Readings (the paper gives no constants):

* grid step S (caller); centre (i, j), i < ceil(W / S), j < ceil(H / S),
  starts at (min(i S + S // 2, W - 1), min(j S + S // 2, H - 1)); index
  j * ceil(W / S) + i;
* a pixel is used when its mask entry is non-zero (no mask: all), its value
  v is finite and |v| < 2048; other pixels get label -1 and D3 = NaN;
* gradient G(x, y) = (v(x+1, y) - v(x-1, y))^2 + (v(x, y+1) - v(x, y-1))^2
  in float64 with coordinates clamped to the image, +inf when one of the
  four pixels is not used; a centre moves to the first position of its 3x3
  neighbourhood (row-major) whose G is strictly below G at the centre, and
  its value is v there (NaN if that pixel is not used: such a centre never
  takes pixels);
* search range: the centres of the 3x3 grid cells around the pixel's cell
  (cell = (x // S, y // S)), tried in index order; distance
  d = (v - v_c)^2 + ((x - x_c)^2 + (y - y_c)^2) w with w = (m / S)^2
  (compactness m), float64, no fused multiply-add; the first smallest wins;
* update: a centre with pixels moves to their mean position and mean value;
  the value mean is taken from v rounded to multiples of 2^-20 and summed
  exactly (integers), so it does not depend on the summation order; a
  centre without pixels stays;
* rounds of assignment then update, at most `iters` of them; the paper
  iterates until the residual between the previous and the updated centres
  converges: here the residual of a round is the largest over the centres
  with pixels of dv^2 + (dx^2 + dy^2) w (the change of the centre in the
  metric of the assignment, float64, no fused multiply-add), and the
  rounds stop after the first whose residual is <= tol^2.  tol = 0 stops
  only when no centre moved, which changes no result (the next round would
  repeat the last one);
* labels are those of the last assignment and D3(p) = v_c of p's centre
  after the last update, rounded to float32.
"""
from __future__ import annotations

import math

import numpy as np

QSCALE = 2.0 ** 20
VMAX = 2048.0


def used(d2, mask=None):
    D = np.asarray(d2, dtype=np.float32).astype(np.float64)
    u = np.isfinite(D) & (np.abs(D) < VMAX)
    if mask is not None:
        u &= np.asarray(mask) != 0
    return D, u


def grid(W, H, S):
    nx, ny = -(-W // S), -(-H // S)
    return nx, ny


def gradient(D, u, x, y):
    H, W = D.shape
    xs = [min(max(x + 1, 0), W - 1), min(max(x - 1, 0), W - 1)]
    ys = [min(max(y + 1, 0), H - 1), min(max(y - 1, 0), H - 1)]
    if not (u[y, xs[0]] and u[y, xs[1]] and u[ys[0], x] and u[ys[1], x]):
        return math.inf
    gx = D[y, xs[0]] - D[y, xs[1]]
    gy = D[ys[0], x] - D[ys[1], x]
    return gx * gx + gy * gy


def init_centres(D, u, S):
    """Centres as float64 arrays (x, y, v)."""
    H, W = D.shape
    nx, ny = grid(W, H, S)
    cx, cy, cv = [], [], []
    for j in range(ny):
        for i in range(nx):
            x0, y0 = min(i * S + S // 2, W - 1), min(j * S + S // 2, H - 1)
            bx, by, best = x0, y0, gradient(D, u, x0, y0)
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    x, y = x0 + dx, y0 + dy
                    if 0 <= x < W and 0 <= y < H:
                        g = gradient(D, u, x, y)
                        if g < best:
                            bx, by, best = x, y, g
            cx.append(float(bx))
            cy.append(float(by))
            cv.append(D[by, bx] if u[by, bx] else math.nan)
    return np.array(cx), np.array(cy), np.array(cv)


def assign(D, u, S, m, cx, cy, cv):
    H, W = D.shape
    nx, ny = grid(W, H, S)
    t = m / S
    w = t * t
    yy, xx = np.mgrid[0:H, 0:W]
    ci, cj = xx // S, yy // S
    best = np.full((H, W), np.inf)
    lab = np.full((H, W), -1, np.int64)
    xf, yf = xx.astype(np.float64), yy.astype(np.float64)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            i, j = ci + di, cj + dj
            ok = (i >= 0) & (i < nx) & (j >= 0) & (j < ny) & u
            k = np.where(ok, j * nx + i, 0)
            dc = D - cv[k]
            ds2 = (xf - cx[k]) ** 2 + (yf - cy[k]) ** 2
            d = dc * dc + ds2 * w
            take = ok & (d < best)
            best = np.where(take, d, best)
            lab = np.where(take, k, lab)
    return lab


def update(D, u, lab, cx, cy, cv):
    H, W = D.shape
    yy, xx = np.mgrid[0:H, 0:W]
    sel = lab >= 0
    k = lab[sel]
    n = len(cx)
    cnt = np.zeros(n, np.int64)
    sx = np.zeros(n, np.int64)
    sy = np.zeros(n, np.int64)
    sq = np.zeros(n, np.int64)
    np.add.at(cnt, k, 1)
    np.add.at(sx, k, xx[sel].astype(np.int64))
    np.add.at(sy, k, yy[sel].astype(np.int64))
    np.add.at(sq, k, np.rint(D[sel] * QSCALE).astype(np.int64))
    has = cnt > 0
    cx, cy, cv = cx.copy(), cy.copy(), cv.copy()
    c = cnt[has].astype(np.float64)
    cx[has] = sx[has].astype(np.float64) / c
    cy[has] = sy[has].astype(np.float64) / c
    cv[has] = (sq[has].astype(np.float64) / c) * (1.0 / QSCALE)
    return cx, cy, cv, cnt


def residual(S, m, old, new, cnt):
    """Largest change of a centre with pixels, dv^2 + (dx^2 + dy^2) w."""
    t = m / S
    w = t * t
    has = cnt > 0
    if not has.any():
        return 0.0
    dx = new[0][has] - old[0][has]
    dy = new[1][has] - old[1][has]
    dv = new[2][has] - old[2][has]
    return float(np.max(dv * dv + (dx * dx + dy * dy) * w))


def slic(d2, S, m, iters, mask=None, tol=0.0, info=None):
    """(labels int64 [H][W], D3 float32 [H][W], centres (x, y, v) float64).
    `info`, a dict, receives "rounds" (the rounds run) and "residuals"."""
    D, u = used(d2, mask)
    cx, cy, cv = init_centres(D, u, S)
    lab = None
    tol2 = tol * tol
    res = []
    for _ in range(iters):
        lab = assign(D, u, S, m, cx, cy, cv)
        nx, ny, nv, cnt = update(D, u, lab, cx, cy, cv)
        res.append(residual(S, m, (cx, cy, cv), (nx, ny, nv), cnt))
        cx, cy, cv = nx, ny, nv
        if res[-1] <= tol2:
            break
    if info is not None:
        info["rounds"] = len(res)
        info["residuals"] = res
    d3 = np.where(lab >= 0, cv[np.maximum(lab, 0)], np.nan).astype(np.float32)
    return lab, d3, (cx, cy, cv)
