"""Seeded synthetic inputs: Gaussian scenes, pinhole camera batches, target images.

This module holds none of the rasterizer's arithmetic. It only draws random
numbers and builds camera poses, and it is the one piece of code that both the
GPU path's tests/benchmarks and the CPU oracle's tests consume. Everything is
numpy (PCG64), float32 unless stated, so the same seed gives the same bytes on
any machine.

The distributions follow the synthetic workloads that stand in for the paper's
datasets (the paper trains on MipNeRF-360 and friends, Sec. 6; none of that data
is used here): means uniform in [-1,1]^3, log-scales normal per axis, normalised
N(0,1) quaternions, sigmoid(N(0,1)) opacities, SH coefficients normal.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

SEED_GAUSSIANS = 0
SEED_CAMERAS = 1
SEED_TARGETS = 2
SEED_REQUESTS = 3


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Scene:
    """Activated Gaussian parameters (float32, row-major, C-contiguous).

    means [P,3]; scales [P,3] (>0); quats [P,4] as (w,x,y,z); opacities [P] in (0,1);
    sh [P,(d+1)^2,3] (coefficient-major, RGB last).
    """
    means: np.ndarray
    scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def P(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(np.ascontiguousarray(self.means[idx]), np.ascontiguousarray(self.scales[idx]),
                     np.ascontiguousarray(self.quats[idx]), np.ascontiguousarray(self.opacities[idx]),
                     np.ascontiguousarray(self.sh[idx]), self.sh_degree)


@dataclass
class Camera:
    """Pinhole camera. R (row-major 3x3) and t map world to camera: x_c = R x_w + t.

    Camera axes: x right, y down, z forward. Pixel (x, y) has its centre at (x+0.5, y+0.5).
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray
    t: np.ndarray
    bg: np.ndarray = field(default_factory=lambda: np.zeros(3, np.float32))


def make_scene(P: int, sh_degree: int, seed: int = SEED_GAUSSIANS, log_scale_mean: float = -4.0,
               log_scale_std: float = 0.5, dc_std: float = 0.3, sh_std: float = 0.2) -> Scene:
    """Draw P Gaussians. At degree 0 the DC coefficients are N(0, dc_std); at degree >= 1 all
    (d+1)^2 x 3 coefficients are N(0, sh_std). Draw order is fixed: means, log-scales, quaternions,
    opacity logits, SH."""
    rng = _rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(P, 3))
    scales = np.exp(rng.normal(log_scale_mean, log_scale_std, size=(P, 3)))
    q = rng.normal(0.0, 1.0, size=(P, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = 1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, size=P)))
    K = (sh_degree + 1) ** 2
    if sh_degree == 0:
        sh = rng.normal(0.0, dc_std, size=(P, 1, 3))
    else:
        sh = rng.normal(0.0, sh_std, size=(P, K, 3))
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f(means), f(scales), f(q), f(opac), f(sh), sh_degree)


def look_at(position: np.ndarray, target=(0.0, 0.0, 0.0)) -> Tuple[np.ndarray, np.ndarray]:
    """World->camera (R, t) for a camera at `position` looking at `target`, world up +y
    (or +z when the view direction is within ~8 degrees of the y axis)."""
    pos = np.asarray(position, np.float64)
    fwd = np.asarray(target, np.float64) - pos
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 1.0, 0.0])
    if abs(float(fwd @ up)) > 0.99:
        up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    t = -R @ pos
    return R, t


def make_camera(width: int, height: int, position, fov_x_deg: float = 60.0, target=(0.0, 0.0, 0.0),
                bg=(0.0, 0.0, 0.0)) -> Camera:
    R, t = look_at(position, target)
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(int(width), int(height), float(np.float32(fx)), float(np.float32(fx)),
                  width / 2.0, height / 2.0, np.ascontiguousarray(R, np.float32),
                  np.ascontiguousarray(t, np.float32), np.asarray(bg, np.float32))


def make_cameras(sizes: Sequence[Tuple[int, int]], seed: int = SEED_CAMERAS, radius=3.0,
                 fov_x_deg: float = 60.0) -> List[Camera]:
    """One camera per (width, height) in `sizes`, positions uniform on a sphere (or a shell when
    `radius` is a (lo, hi) pair) around the origin, all looking at the origin."""
    rng = _rng(seed)
    cams = []
    for (w, h) in sizes:
        d = rng.normal(0.0, 1.0, size=3)
        d /= np.linalg.norm(d)
        if isinstance(radius, (tuple, list)):
            r = rng.uniform(radius[0], radius[1])
        else:
            r = float(radius)
        cams.append(make_camera(w, h, d * r, fov_x_deg))
    return cams


def make_targets(cams: Sequence[Camera], seed: int = SEED_TARGETS) -> List[np.ndarray]:
    """Target images [3,H,W] float32, U[0,1]."""
    rng = _rng(seed)
    return [np.ascontiguousarray(rng.uniform(0.0, 1.0, size=(3, c.height, c.width)), np.float32) for c in cams]


# ---------------------------------------------------------------------------------------------
# The five synthetic workloads. Sizes and distributions are those of the benchmark configurations
# (the paper's datasets are not used; these stand in for them).
# ---------------------------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    P: int
    sh_degree: int
    sizes: List[Tuple[int, int]]
    radius: object = 3.0
    log_scale_mean: float = -4.0
    log_scale_std: float = 0.5
    w_l1: float = 1.0
    w_dssim: float = 0.0
    densify: bool = False
    tile: Tuple[int, int] = (16, 16)

    def scene(self) -> Scene:
        return make_scene(self.P, self.sh_degree, log_scale_mean=self.log_scale_mean,
                          log_scale_std=self.log_scale_std)

    def cameras(self) -> List[Camera]:
        return make_cameras(self.sizes, radius=self.radius)


WORKLOADS = {
    "small_16k_4x128": Workload("small_16k_4x128", 16384, 0, [(128, 128)] * 4),
    "train_300k_4x1600x1064_dssim": Workload("train_300k_4x1600x1064_dssim", 300_000, 3, [(1600, 1064)] * 4,
                                             w_l1=0.8, w_dssim=0.2),
    "uneven_1m_8view": Workload("uneven_1m_8view", 1_000_000, 3,
                                [(1920, 1080)] * 3 + [(1280, 720)] * 3 + [(980, 545)] * 2,
                                radius=(2.5, 4.0)),
    "large_3m_16x1280x840": Workload("large_3m_16x1280x840", 3_000_000, 3, [(1280, 840)] * 16,
                                     log_scale_mean=-5.0, log_scale_std=0.7, densify=True),
}

SERVE_RESOLUTIONS = [(256, 256), (640, 480), (1280, 720), (1920, 1080)]


def make_requests(n: int, rate_hz: float = 200.0, seed: int = SEED_REQUESTS,
                  resolutions: Sequence[Tuple[int, int]] = SERVE_RESOLUTIONS, radius: float = 3.0):
    """A seeded stream of `n` render requests: Poisson arrivals at `rate_hz` (exponential gaps,
    first arrival after one gap; rate 0 or inf puts every arrival at 0), a resolution drawn
    uniformly from `resolutions`, and a camera on a sphere of `radius` looking at the origin.
    Returns (arrival seconds [n] float64, list of Camera)."""
    rng = _rng(seed)
    if rate_hz and math.isfinite(rate_hz):
        arrivals = np.cumsum(rng.exponential(1.0 / rate_hz, size=n))
    else:
        arrivals = np.zeros(n)
    which = rng.integers(0, len(resolutions), size=n)
    cams = []
    for i in range(n):
        d = rng.normal(0.0, 1.0, size=3)
        d /= np.linalg.norm(d)
        w, h = resolutions[int(which[i])]
        cams.append(make_camera(w, h, d * radius))
    return arrivals, cams
