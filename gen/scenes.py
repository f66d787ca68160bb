"""Seeded scene / camera / text / target generators.

Distributions follow the synthetic workloads that stand in for the paper's
LERF scenes (the paper's own scenes, trained Gaussians and CLIP features are not
available): means uniform in [-1,1]^3, log-scales N(-4, 0.5), uniformly random
unit quaternions, opacity sigmoid(N(0,1)), K distinct atom indices per
Gaussian and semantic level with softmax(N(0,1)) weights (so each code sums to
one, as the sparse code of Section 3.3 requires), and an L x D dictionary with
unit-norm N(0,1) rows.  Everything is drawn in float64 from one
``numpy.random.default_rng(seed)`` in a fixed order and cast to float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Camera:
    """Pinhole camera, OpenCV axes (x right, y down, z forward).

    Pixel (px, py) is sampled at (px + 0.5, py + 0.5).  ``world_to_cam`` is
    the 3x4 row-major [R | t] mapping world points to camera space.
    """
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    world_to_cam: np.ndarray  # (3, 4) float32
    znear: float = 0.2

    def as_array(self) -> np.ndarray:
        """Flat float64 view: [W, H, fx, fy, cx, cy, R00..R22, t0..t2, znear]."""
        r = self.world_to_cam.astype(np.float64)
        return np.array([self.width, self.height, self.fx, self.fy, self.cx, self.cy,
                         *r[:, :3].reshape(-1), *r[:, 3], self.znear], dtype=np.float64)

    @property
    def tiles_x(self) -> int:
        return (self.width + 15) // 16

    @property
    def tiles_y(self) -> int:
        return (self.height + 15) // 16


def _focal_from_hfov(width: int, fov_x_deg: float) -> float:
    return float(np.float32((width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)))


def make_camera(width: int, height: int, fov_x_deg: float = 60.0, distance: float = 3.0) -> Camera:
    """Camera at (0, 0, -distance) looking at the origin along +z (R = I)."""
    f = _focal_from_hfov(width, fov_x_deg)
    w2c = np.zeros((3, 4), dtype=np.float32)
    w2c[:, :3] = np.eye(3, dtype=np.float32)
    w2c[2, 3] = distance
    return Camera(width, height, f, f, width / 2.0, height / 2.0, w2c)


def orbit_camera(width: int, height: int, view: int, n_views: int = 8,
                 radius: float = 3.0, fov_x_deg: float = 60.0) -> Camera:
    """View ``view`` of ``n_views`` on a horizontal circle of ``radius``
    around the origin, each looking at the origin."""
    th = 2.0 * math.pi * view / n_views
    rot = np.array([[math.cos(th), 0.0, math.sin(th)],
                    [0.0, 1.0, 0.0],
                    [-math.sin(th), 0.0, math.cos(th)]])
    center = radius * np.array([math.sin(th), 0.0, -math.cos(th)])
    t = -rot @ center
    w2c = np.zeros((3, 4), dtype=np.float32)
    w2c[:, :3] = rot
    w2c[:, 3] = t
    f = _focal_from_hfov(width, fov_x_deg)
    return Camera(width, height, f, f, width / 2.0, height / 2.0, w2c)


@dataclass
class Scene:
    means: np.ndarray      # (N, 3) f32
    scales: np.ndarray     # (N, 3) f32, > 0
    quats: np.ndarray      # (N, 4) f32, (w, x, y, z), unit norm
    opacity: np.ndarray    # (N,) f32 in (0, 1)
    topk_idx: np.ndarray   # (N, levels, K) i32 in [0, L)
    topk_w: np.ndarray     # (N, levels, K) f32
    dictionary: np.ndarray  # (L, D) f32
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.means.shape[0]

    @property
    def levels(self) -> int:
        return self.topk_idx.shape[1]

    @property
    def K(self) -> int:
        return self.topk_idx.shape[2]

    @property
    def L(self) -> int:
        return self.dictionary.shape[0]

    @property
    def D(self) -> int:
        return self.dictionary.shape[1]


def _softmax_rows(x: np.ndarray) -> np.ndarray:
    e = np.exp(x - x.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def make_scene(seed: int, n: int, L: int = 64, K: int = 4, D: int = 512, levels: int = 1,
               mean_range: float = 1.0, log_scale_mu: float = -4.0, log_scale_sigma: float = 0.5) -> Scene:
    """Draw one scene.  Draw order: means, log-scales, quaternions, opacity
    logits, then per level (index keys, weight logits), then the dictionary."""
    if K > L:
        raise ValueError("K must not exceed L")
    rng = np.random.default_rng(seed)
    means = rng.uniform(-mean_range, mean_range, size=(n, 3))
    scales = np.exp(rng.normal(log_scale_mu, log_scale_sigma, size=(n, 3)))
    q = rng.normal(0.0, 1.0, size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opacity = 1.0 / (1.0 + np.exp(-rng.normal(0.0, 1.0, size=n)))
    idx = np.empty((n, levels, K), dtype=np.int32)
    w = np.empty((n, levels, K), dtype=np.float64)
    for lv in range(levels):
        keys = rng.random(size=(n, L))
        idx[:, lv, :] = np.argsort(keys, axis=1, kind="stable")[:, :K]
        w[:, lv, :] = _softmax_rows(rng.normal(0.0, 1.0, size=(n, K)))
    dic = rng.normal(0.0, 1.0, size=(L, D))
    dic /= np.linalg.norm(dic, axis=1, keepdims=True)
    return Scene(means.astype(np.float32), scales.astype(np.float32), q.astype(np.float32),
                 opacity.astype(np.float32), idx, w.astype(np.float32), dic.astype(np.float32))


def make_text(seed: int, D: int = 512, n_neg: int = 4):
    """One positive and ``n_neg`` canonical negative unit-norm embeddings."""
    rng = np.random.default_rng(seed)
    e = rng.normal(0.0, 1.0, size=(1 + n_neg, D))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    e = e.astype(np.float32)
    return e[0].copy(), e[1:].copy()


def make_target_factors(seed: int, height: int, width: int, D: int = 512, rank: int = 8):
    """Smooth random target field Y = up(Z) @ P.

    Z ~ N(0,1) on a (ceil(H/64)+1) x (ceil(W/64)+1) x rank grid, bilinearly
    upsampled (align-corners) to H x W x rank; P ~ N(0,1)^(rank x D) / sqrt(rank).
    Returns (Zup (H, W, rank) f32, P (rank, D) f32).
    """
    rng = np.random.default_rng(seed)
    gh, gw = -(-height // 64) + 1, -(-width // 64) + 1
    z = rng.normal(0.0, 1.0, size=(gh, gw, rank))
    p = rng.normal(0.0, 1.0, size=(rank, D)) / math.sqrt(rank)
    ys = np.linspace(0.0, gh - 1, height)
    xs = np.linspace(0.0, gw - 1, width)
    y0 = np.minimum(np.floor(ys).astype(np.int64), gh - 2)
    x0 = np.minimum(np.floor(xs).astype(np.int64), gw - 2)
    fy = (ys - y0)[:, None, None]
    fx = (xs - x0)[None, :, None]
    z00 = z[y0][:, x0]
    z01 = z[y0][:, x0 + 1]
    z10 = z[y0 + 1][:, x0]
    z11 = z[y0 + 1][:, x0 + 1]
    up = (1 - fy) * ((1 - fx) * z00 + fx * z01) + fy * ((1 - fx) * z10 + fx * z11)
    return up.astype(np.float32), p.astype(np.float32)


def target_map(zup: np.ndarray, p: np.ndarray) -> np.ndarray:
    """Materialise Y = Zup @ P as float32 (H, W, D), accumulating in float64."""
    h, w, r = zup.shape
    y = zup.reshape(-1, r).astype(np.float64) @ p.astype(np.float64)
    return y.astype(np.float32).reshape(h, w, -1)


# Workload configurations (synthetic stand-ins for the paper's LERF scenes).
CONFIGS = {
    # small parity case: 2k Gaussians, 128x128
    "c1": dict(seed=1001, n=2000, width=128, height=128, L=64, K=4, D=512, levels=1),
    # headline feature-map/query workload: 300k Gaussians at 1440x1080
    "c2": dict(seed=1002, n=300_000, width=1440, height=1080, L=64, K=4, D=512, levels=1),
    # differentiation workload (same scene shape as c2)
    "c3": dict(seed=1003, n=300_000, width=1440, height=1080, L=64, K=4, D=512, levels=1),
    # precision sweep base (L, K overridden per case)
    "c4": dict(seed=1004, n=300_000, width=1440, height=1080, L=64, K=4, D=512, levels=1),
    # full form: 1M Gaussians, 1920x1080, 3 levels, 8 orbit views
    "c5": dict(seed=1005, n=1_000_000, width=1920, height=1080, L=64, K=4, D=512, levels=3),
    # finite-difference scene: 500 Gaussians at 64x64
    "fd": dict(seed=1100, n=500, width=64, height=64, L=64, K=4, D=512, levels=1),
}


def config_scene(name: str, **overrides):
    """(Scene, Camera) for a named configuration; keyword overrides replace
    entries of the configuration (e.g. ``n=`` for a reduced sample)."""
    c = dict(CONFIGS[name])
    c.update(overrides)
    scene = make_scene(c["seed"], c["n"], L=c["L"], K=c["K"], D=c["D"], levels=c["levels"])
    cam = make_camera(c["width"], c["height"])
    return scene, cam
