"""Seeded synthetic road stereo pairs (input generator only).

The paper evaluates on KITTI road regions and on its own pothole datasets;
neither is available, so every workload here is generated.  This module
renders a rectified uint8 pair of a textured road plane seen by a pitched
and rolled stereo rig, with two smooth elliptical pothole depressions, and
returns the exact disparity of every left pixel.

It holds none of the matching arithmetic (census, cost, aggregation,
winner-take-all, sub-pixel): it only draws images.  Both the HIP path and
the CPU oracle receive the arrays it returns.

Scene model
-----------
* Principal point at the image centre ``(cx, cy) = ((W-1)/2, (H-1)/2)``.
* Baseline ``b``, camera height ``h``, pitch ``theta``, roll ``phi``.
* On the road plane the disparity of the left pixel ``(u, v)`` is the
  roll-aware v-disparity line of Sec. II-A, eq. (3), written in centred
  coordinates:  ``d = a0 + a1 * (cos(phi)*(v-cy) - sin(phi)*(u-cx))`` with
  ``a1 = (b/h) cos(theta)`` and ``a0 = (b/h) f sin(theta)``.
* Where that value is below 0.5 px (above the horizon) the scene is a far
  background at disparity 0.
* Inside a pothole of depth ``z`` (metres, paraboloid profile) the road
  point lies deeper, and its disparity becomes ``d * h / (h + z)``.
* Texture: fractal gradient ("improved Perlin") noise evaluated in
  continuous image coordinates, 6 octaves, base wavelength 32 px, gain
  0.5, intensity 128 with a standard deviation of about 40 (clamped).
* Left image: texture + N(0, sigma^2), rounded to uint8.
* Right image: for each right pixel ``x`` the matching left position
  solves ``u = x + d(u, v)``, found by 3 fixed-point iterations from
  ``u = x``; the clean texture is evaluated there, independent noise is
  added and the result rounded.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = ["RoadScene", "make_pair", "make_pair_torch", "scene_for_config", "PairSet",
           "CONFIGS", "road_model_disparity"]


@dataclasses.dataclass(frozen=True)
class RoadScene:
    width: int
    height: int
    focal: float = 900.0
    baseline: float = 0.1
    cam_height: float = 1.0
    pitch_deg: float = 5.0
    roll_deg: float = 0.0
    noise_sigma: float = 2.0
    n_potholes: int = 2
    depth_range: tuple = (0.03, 0.08)
    octaves: int = 6
    base_wavelength: float = 32.0
    gain: float = 0.5
    contrast: float = 40.0

    @property
    def cx(self) -> float:
        return (self.width - 1) / 2.0

    @property
    def cy(self) -> float:
        return (self.height - 1) / 2.0

    @property
    def road_params(self):
        """(a0, a1, phi) of the road line in centred coordinates."""
        th = math.radians(self.pitch_deg)
        k = self.baseline / self.cam_height
        return (k * self.focal * math.sin(th), k * math.cos(th),
                math.radians(self.roll_deg))


def road_model_disparity(a0, a1, phi, u, v, cx, cy):
    """Road-plane disparity at (u, v): the scene's ground truth on the road."""
    return a0 + a1 * (math.cos(phi) * (v - cy) - math.sin(phi) * (u - cx))


# ---------------------------------------------------------------------------
# gradient noise


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


class _GradientNoise:
    """One octave of 2-D gradient noise on a random lattice (seeded)."""

    def __init__(self, rng: np.random.Generator, period: int = 256):
        self.period = period
        ang = rng.uniform(0.0, 2.0 * math.pi, size=(period, period))
        self.gx = np.cos(ang)
        self.gy = np.sin(ang)
        self.off = rng.uniform(0.0, 1.0, size=2)

    def __call__(self, x, y):
        x = x + self.off[0]
        y = y + self.off[1]
        x0 = np.floor(x)
        y0 = np.floor(y)
        fx = x - x0
        fy = y - y0
        p = self.period
        ix = x0.astype(np.int64) % p
        iy = y0.astype(np.int64) % p
        ix1 = (ix + 1) % p
        iy1 = (iy + 1) % p

        def dot(jx, jy, dx, dy):
            return self.gx[jy, jx] * dx + self.gy[jy, jx] * dy

        n00 = dot(ix, iy, fx, fy)
        n10 = dot(ix1, iy, fx - 1.0, fy)
        n01 = dot(ix, iy1, fx, fy - 1.0)
        n11 = dot(ix1, iy1, fx - 1.0, fy - 1.0)
        sx = _fade(fx)
        sy = _fade(fy)
        a = n00 + sx * (n10 - n00)
        b = n01 + sx * (n11 - n01)
        return a + sy * (b - a)


class _Texture:
    def __init__(self, scene: RoadScene, rng: np.random.Generator):
        self.octs = [_GradientNoise(rng) for _ in range(scene.octaves)]
        self.scene = scene

    def __call__(self, x, y):
        s = self.scene
        acc = np.zeros(np.broadcast(x, y).shape)
        amp = 1.0
        norm = 0.0
        wl = s.base_wavelength
        for o in self.octs:
            acc += amp * o(x / wl, y / wl)
            norm += amp
            amp *= s.gain
            wl = max(wl / 2.0, 1.0)
        # the normalised fractal sum has a standard deviation of about 0.2;
        # scale it so that one standard deviation is `contrast` grey levels
        return np.clip(128.0 + s.contrast * (acc / norm) / 0.2, 0.0, 255.0)


# ---------------------------------------------------------------------------
# scene geometry


def _potholes(scene: RoadScene, rng: np.random.Generator):
    """Ellipses (cu, cv, ru, rv, depth) placed on the road below the horizon."""
    a0, a1, phi = scene.road_params
    horizon = scene.cy - a0 / a1  # row where the road disparity reaches 0
    top = max(horizon + 0.25 * (scene.height - horizon), 0.0)
    out = []
    for _ in range(scene.n_potholes):
        ru = rng.uniform(0.06, 0.12) * scene.width
        rv = rng.uniform(0.04, 0.08) * scene.height
        cu = rng.uniform(ru, scene.width - 1 - ru)
        cv = rng.uniform(min(top + rv, scene.height - 1 - rv),
                         scene.height - 1 - rv)
        depth = rng.uniform(*scene.depth_range)
        out.append((cu, cv, ru, rv, depth))
    return out


def _disparity(scene: RoadScene, holes, u, v):
    """Exact disparity of the left pixel at continuous (u, v)."""
    a0, a1, phi = scene.road_params
    d = road_model_disparity(a0, a1, phi, u, v, scene.cx, scene.cy)
    d = np.asarray(d, dtype=np.float64)
    road = d >= 0.5
    z = np.zeros_like(d)
    for cu, cv, ru, rv, depth in holes:
        r2 = ((u - cu) / ru) ** 2 + ((v - cv) / rv) ** 2
        z = np.maximum(z, np.where(r2 < 1.0, depth * (1.0 - r2), 0.0))
    d = np.where(road, d * scene.cam_height / (scene.cam_height + z), 0.0)
    return d, road, road & (z > 0.0)


@dataclasses.dataclass
class PairSet:
    left: np.ndarray        # uint8 [H, W]
    right: np.ndarray       # uint8 [H, W]
    gt: np.ndarray          # float64 [H, W] disparity of each left pixel
    road: np.ndarray        # bool [H, W] road (not background) pixels
    pothole: np.ndarray     # bool [H, W] pixels inside a depression
    road_params: tuple      # (a0, a1, phi) in centred coordinates
    centre: tuple           # (cx, cy)
    scene: RoadScene


def make_pair(scene: RoadScene, seed: int) -> PairSet:
    """Render one seeded pair."""
    rng = np.random.default_rng(seed)
    tex = _Texture(scene, rng)
    holes = _potholes(scene, rng)
    H, W = scene.height, scene.width
    vv, uu = np.mgrid[0:H, 0:W].astype(np.float64)
    gt, road, hole = _disparity(scene, holes, uu, vv)
    clean_l = tex(uu, vv)
    # right pixel x sees the left point u with u - d(u, v) = x
    u = uu.copy()
    for _ in range(3):
        u = uu + _disparity(scene, holes, u, vv)[0]
    clean_r = tex(u, vv)
    nl = rng.normal(0.0, scene.noise_sigma, size=(H, W))
    nr = rng.normal(0.0, scene.noise_sigma, size=(H, W))
    left = np.clip(np.rint(clean_l + nl), 0, 255).astype(np.uint8)
    right = np.clip(np.rint(clean_r + nr), 0, 255).astype(np.uint8)
    return PairSet(left, right, gt, road, hole, scene.road_params,
                   (scene.cx, scene.cy), scene)


# ---------------------------------------------------------------------------
# the same scenes rendered with torch (on the GPU, for training data)


def _noise_torch(o: _GradientNoise, x, y, gx, gy):
    import torch
    x = x + float(o.off[0])
    y = y + float(o.off[1])
    x0 = torch.floor(x)
    y0 = torch.floor(y)
    fx = x - x0
    fy = y - y0
    p = o.period
    ix = x0.long() % p
    iy = y0.long() % p
    ix1 = (ix + 1) % p
    iy1 = (iy + 1) % p

    def dot(jx, jy, dx, dy):
        k = jy * p + jx
        return gx[k] * dx + gy[k] * dy

    n00 = dot(ix, iy, fx, fy)
    n10 = dot(ix1, iy, fx - 1.0, fy)
    n01 = dot(ix, iy1, fx, fy - 1.0)
    n11 = dot(ix1, iy1, fx - 1.0, fy - 1.0)
    sx = _fade(fx)
    sy = _fade(fy)
    a = n00 + sx * (n10 - n00)
    b = n01 + sx * (n11 - n01)
    return a + sy * (b - a)


def make_pair_torch(scene: RoadScene, seed: int, device="cuda", noise=True):
    """The scene of make_pair(scene, seed) rendered with torch in float64 on
    `device`: same lattices, potholes and formulas, so the clean images and
    the ground truth agree with make_pair's; the sensor noise is drawn from
    torch's generator (same distribution, other samples).  Returns
    (left, right, gt, road) tensors: uint8, uint8, float32, bool."""
    import torch
    rng = np.random.default_rng(seed)
    tex = _Texture(scene, rng)
    holes = _potholes(scene, rng)
    H, W = scene.height, scene.width
    dev = torch.device(device)
    f64 = torch.float64
    vv = torch.arange(H, dtype=f64, device=dev)[:, None].expand(H, W)
    uu = torch.arange(W, dtype=f64, device=dev)[None, :].expand(H, W)
    lat = [(torch.from_numpy(o.gx.ravel()).to(dev), torch.from_numpy(o.gy.ravel()).to(dev))
           for o in tex.octs]
    a0, a1, phi = scene.road_params

    def disparity(u, v):
        d = a0 + a1 * (math.cos(phi) * (v - scene.cy) - math.sin(phi) * (u - scene.cx))
        road = d >= 0.5
        z = torch.zeros_like(d)
        for cu, cv, ru, rv, depth in holes:
            r2 = ((u - cu) / ru) ** 2 + ((v - cv) / rv) ** 2
            z = torch.maximum(z, torch.where(r2 < 1.0, depth * (1.0 - r2), torch.zeros_like(r2)))
        return torch.where(road, d * scene.cam_height / (scene.cam_height + z), torch.zeros_like(d)), road

    def texture(x, y):
        acc = torch.zeros_like(x)
        amp, norm, wl = 1.0, 0.0, scene.base_wavelength
        for o, (gx, gy) in zip(tex.octs, lat):
            acc = acc + amp * _noise_torch(o, x / wl, y / wl, gx, gy)
            norm += amp
            amp *= scene.gain
            wl = max(wl / 2.0, 1.0)
        return torch.clamp(128.0 + scene.contrast * (acc / norm) / 0.2, 0.0, 255.0)

    gt, road = disparity(uu, vv)
    clean_l = texture(uu, vv)
    u = uu.clone()
    for _ in range(3):
        u = uu + disparity(u, vv)[0]
    clean_r = texture(u, vv)
    if noise:
        g = torch.Generator(device=dev)
        g.manual_seed(int(seed))
        clean_l = clean_l + scene.noise_sigma * torch.randn((H, W), generator=g, dtype=f64, device=dev)
        clean_r = clean_r + scene.noise_sigma * torch.randn((H, W), generator=g, dtype=f64, device=dev)
    left = torch.clamp(torch.round(clean_l), 0, 255).to(torch.uint8)
    right = torch.clamp(torch.round(clean_r), 0, 255).to(torch.uint8)
    return left, right, gt.to(torch.float32), road


# ---------------------------------------------------------------------------
# the workloads


CONFIGS = {
    # 320x240, census 5x5, 4 paths, disparities 0..31, roll 2 deg
    "road320": dict(width=320, height=240, focal=300.0, roll=2.0,
                    census=5, ndisp=32, npaths=4, p1=10, p2=120),
    # 1280x720, census 7x7, 8 paths, disparities 0..127, roll U(0,3) deg
    "road1280": dict(width=1280, height=720, focal=900.0, roll=(0.0, 3.0),
                     census=7, ndisp=128, npaths=8, p1=10, p2=120),
    # 1280x720, per-row windows of width 24 from the road model
    "road1280_pt": dict(width=1280, height=720, focal=900.0, roll=(0.0, 3.0),
                        census=7, ndisp=24, npaths=8, p1=10, p2=120),
    # 1920x1080 full range 0..191 (learned-window workload)
    "road1920": dict(width=1920, height=1080, focal=1350.0, roll=(0.0, 4.0),
                     census=7, ndisp=192, npaths=8, p1=10, p2=120),
    # 640x480 disparities 0..63 (batched workload member)
    "road640": dict(width=640, height=480, focal=450.0, roll=(0.0, 4.0),
                    census=7, ndisp=64, npaths=8, p1=10, p2=120),
}


def scene_for_config(name: str, seed: int) -> RoadScene:
    c = CONFIGS[name]
    roll = c["roll"]
    if isinstance(roll, tuple):
        roll = float(np.random.default_rng(seed ^ 0x5EED).uniform(*roll))
    return RoadScene(width=c["width"], height=c["height"], focal=c["focal"],
                     roll_deg=roll)
