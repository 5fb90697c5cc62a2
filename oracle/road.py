"""CPU oracle of the road model and the disparity transformation
(test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It shares no code with the HIP path.

Road model (Sec. II-A, eq. (3)): on the road the disparity of pixel
p = (u, v) is f(a, p, phi) = a0 + a1 (v cos(phi) - u sin(phi)), with the
roll rotation taken about the image centre, i.e. u and v measured from
(cx, cy) = ((W-1)/2, (H-1)/2).

Fit (Sec. II-C): over the k selected pixels, eq. (5) defines
E0(a, phi) = |d - T(phi) a|^2 with T(phi) = [1_k, cos(phi) v - sin(phi) u];
eq. (11) gives the best a for a fixed phi and eq. (12) the residual
E0min(phi) that remains.  The paper minimises E0min over phi with a method
it cites but does not print; this oracle searches phi directly: E0min
(evaluated as the residual of eq. (5) at eq. (11), which eq. (12) expands)
on a grid of 1-degree steps over (-90, 90] degrees (E0min has period 180
degrees, since T(phi + 180) spans the same columns), then a golden-section
search in the two grid steps around the best grid point.  a follows from
eq. (11) at the phi found.

Disparity transformation (Sec. II-C, eq. (13)):
D2(p) = D1(p) - f(a, p, phi) + delta_DT.

Road region without ground truth (the paper selects it by hand): pixels
whose road disparity f(a, p, phi) is at least f_min, i.e. below the horizon
line of the fitted road, where the road's match lies inside the right image
(u - f >= margin; left of that band no disparity can be measured), with a
finite disparity.

Pixel selection (the paper fits "road disparities" without saying how they
are chosen): a pixel (column u, row v, integer indices) is used when its
mask entry is non-zero (no mask: all pixels), its disparity d is finite and
at least `min_disp`, and its match lies inside the right image with room to
spare: u - d >= `margin` (computed in float64).  A refit keeps only the
pixels within `tol` of an earlier fit's road line, the "road disparities"
of Sec. II-C being those on the road plane (the background and other
outliers bias a plain least-squares fit).

Status: 0 fitted; 1 fewer than 3 pixels selected; 2 the selected pixels lie
on one image line (the 2x2 covariance of (u, v) has
det <= 1e-9 * var(u) * var(v)), where eq. (11) has no unique solution for
every phi.  a0, a1, phi and E0min are NaN unless the status is 0.

Everything is float64 numpy; the matrix products and the 2x2 solves are
library routines, nothing is blocked or reordered.
"""
from __future__ import annotations

import math

import numpy as np

GRID_STEPS = 180            # grid over (-pi/2, pi/2]
GOLDEN_TOL = 1e-11          # final bracket width of the golden-section search (rad)
COLLINEAR = 1e-9


def select(disp, mask=None, min_disp=-math.inf, margin=-math.inf, prior=None, tol=math.inf):
    """Centred coordinates (u, v) and disparities d (float64) of the pixels
    that enter the fit; `prior` = (a0, a1, phi) of an earlier fit keeps only
    the pixels within `tol` of its road line."""
    D = np.asarray(disp)
    H, W = D.shape
    cols = np.arange(W, dtype=np.float64)[None, :]
    keep = np.isfinite(D) & (D >= min_disp) & (cols - D.astype(np.float64) >= margin)
    if prior is not None:
        keep &= np.abs(D.astype(np.float64) - road_disparity(*prior, W, H)) <= tol
    if mask is not None:
        keep &= np.asarray(mask) != 0
    vv, uu = np.nonzero(keep)
    u = uu.astype(np.float64) - (W - 1) / 2.0
    v = vv.astype(np.float64) - (H - 1) / 2.0
    return u, v, D[keep].astype(np.float64)


def T_matrix(u, v, phi):
    """T(phi) of Sec. II-A: columns 1_k and cos(phi) v - sin(phi) u."""
    return np.stack([np.ones_like(u), math.cos(phi) * v - math.sin(phi) * u], axis=1)


def a_of_phi(u, v, d, phi):
    """eq. (11): a(phi) = (T^T T)^-1 T^T d."""
    T = T_matrix(u, v, phi)
    return np.linalg.solve(T.T @ T, T.T @ d)


def e0min(u, v, d, phi):
    """eq. (12): E0min(phi) = d^T d - d^T T (T^T T)^-1 T^T d."""
    T = T_matrix(u, v, phi)
    Td = T.T @ d
    return float(d @ d - Td @ np.linalg.solve(T.T @ T, Td))


def residual(u, v, d, phi):
    """eq. (5) at a = a(phi) of eq. (11): |d - T(phi) a(phi)|^2, the same
    quantity as eq. (12) without its cancellation between d^T d and the
    projected part (used by the search)."""
    r = d - T_matrix(u, v, phi) @ a_of_phi(u, v, d, phi)
    return float(r @ r)


def _wrap(phi):
    """phi modulo pi into (-pi/2, pi/2]."""
    phi = phi - math.pi * round(phi / math.pi)
    return math.pi / 2 if phi <= -math.pi / 2 else phi


def minimise_phi(u, v, d):
    """phi in (-pi/2, pi/2] minimising E0min (evaluated as the residual of
    eq. (5) at eq. (11)): grid, then golden section."""
    step = math.pi / GRID_STEPS
    grid = [-math.pi / 2 + i * step for i in range(1, GRID_STEPS + 1)]
    vals = [residual(u, v, d, p) for p in grid]
    best = grid[int(np.argmin(vals))]
    lo, hi = best - step, best + step
    g = (math.sqrt(5.0) - 1.0) / 2.0
    x1, x2 = hi - g * (hi - lo), lo + g * (hi - lo)
    f1, f2 = residual(u, v, d, x1), residual(u, v, d, x2)
    while hi - lo > GOLDEN_TOL:
        if f1 <= f2:
            hi, x2, f2 = x2, x1, f1
            x1 = hi - g * (hi - lo)
            f1 = residual(u, v, d, x1)
        else:
            lo, x1, f1 = x1, x2, f2
            x2 = lo + g * (hi - lo)
            f2 = residual(u, v, d, x2)
    return _wrap(0.5 * (lo + hi))


def fit_road(disp, mask=None, min_disp=-math.inf, margin=-math.inf, prior=None, tol=math.inf):
    """Fit of Sec. II-C to one disparity map [H][W]: dict with status, count,
    a0, a1, phi (radians) and e0min.  With `prior` ((a0, a1, phi), or None)
    only pixels within `tol` of the prior road line enter (the refit)."""
    u, v, d = select(disp, mask, min_disp, margin, prior, tol)
    k = d.size
    nan = float("nan")
    out = dict(status=0, count=k, a0=nan, a1=nan, phi=nan, e0min=nan)
    if k < 3:
        out["status"] = 1
        return out
    uc, vc = u - u.mean(), v - v.mean()
    cuu, cvv, cuv = float(uc @ uc), float(vc @ vc), float(uc @ vc)
    if not cuu * cvv - cuv * cuv > COLLINEAR * cuu * cvv:
        out["status"] = 2
        return out
    phi = minimise_phi(u, v, d)
    a = a_of_phi(u, v, d, phi)
    out.update(a0=float(a[0]), a1=float(a[1]), phi=phi, e0min=residual(u, v, d, phi))
    return out


def road_disparity(a0, a1, phi, W, H):
    """eq. (3) at every pixel, float64 [H][W], centred coordinates."""
    v, u = np.mgrid[0:H, 0:W].astype(np.float64)
    return a0 + a1 * (math.cos(phi) * (v - (H - 1) / 2.0) - math.sin(phi) * (u - (W - 1) / 2.0))


def transform(disp, a0, a1, phi, delta_dt):
    """eq. (13): D2 = D1 - f(a, p, phi) + delta_DT, in float64, returned as
    float32."""
    D1 = np.asarray(disp, dtype=np.float64)
    H, W = D1.shape
    return (D1 - road_disparity(a0, a1, phi, W, H) + delta_dt).astype(np.float32)


def road_mask(disp, a0, a1, phi, f_min, margin):
    """Road region used without ground truth: pixels where the road line of
    eq. (3) is at least f_min (below the horizon line) and its match lies at
    least `margin` inside the right image (u - f >= margin), with a finite
    disparity; uint8 [H][W]."""
    D = np.asarray(disp, dtype=np.float32).astype(np.float64)
    H, W = D.shape
    f = road_disparity(a0, a1, phi, W, H)
    cols = np.arange(W, dtype=np.float64)[None, :]
    return ((f >= f_min) & (cols - f >= margin) & np.isfinite(D)).astype(np.uint8)


def window_map(a0, a1, phi, W, H, w, scale=1.0):
    """Per-pixel windows centred on the road plane of eq. (3) (a0 of a fit
    at 1/scale resolution scaled by `scale`): lo = max(0, floor(f + 1/2) -
    floor(w/2)), int32 [H][W]."""
    f = road_disparity(scale * a0, a1, phi, W, H)
    lo = np.floor(f + 0.5) - (w // 2)
    return np.where(lo > 0, lo, 0).astype(np.int32)
