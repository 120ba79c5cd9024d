"""Seeded synthetic inputs shared by the oracle, the GPU path, the tests and the benchmark.

This module holds input recipes only: random draws, cameras and workload shapes. It holds
none of the rasterizer's arithmetic (no projection, compositing or gradients), so the oracle
and the HIP path can both read what it produces without sharing any method code.

Every draw uses ``numpy.random.Generator(PCG64(seed))`` in float64 and is cast to float32 once.
The MipNeRF360 scenes and pretrained models the paper measures on (Sec. 4) are not available;
these generators stand in for them with the shapes, sizes and value distributions of the
workloads named in the task configuration (2D splats; clustered 3D scenes; ring cameras;
a serving mix of scene sizes and resolutions).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Camera", "Scene", "Splats2D", "rng", "splats2d", "scene3d", "camera_front",
    "camera_ring", "image_grad", "sorted_key_case", "serving_scenes", "serving_requests",
    "CFG1", "CFG2", "CFG3", "CFG4", "CFG5_RESOLUTIONS",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclasses.dataclass
class Camera:
    """Pinhole camera. ``viewmat`` is the 3x4 world->camera matrix [R|t] (row-major);
    the camera looks along +z with x to the right and y down (pixel units)."""
    viewmat: np.ndarray  # (3, 4) float32
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.2

    @property
    def campos(self) -> np.ndarray:
        R = self.viewmat[:, :3].astype(np.float64)
        t = self.viewmat[:, 3].astype(np.float64)
        return -R.T @ t


@dataclasses.dataclass
class Scene:
    """3D Gaussians, already activated: positive scales, opacity in (0, 1), raw quaternions
    (w, x, y, z) that the projection normalises, SH coefficients [N, K, 3]."""
    means3d: np.ndarray   # (N, 3) float32
    scales: np.ndarray    # (N, 3) float32
    quats: np.ndarray     # (N, 4) float32
    opacities: np.ndarray  # (N,) float32
    sh: np.ndarray        # (N, K, 3) float32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means3d.shape[0])


@dataclasses.dataclass
class Splats2D:
    """Pre-projected splats: means in pixels, conic (a, b, c) of the inverse 2D covariance
    with q = a dx^2 + 2 b dx dy + c dy^2, opacity, colour and depth."""
    means2d: np.ndarray   # (N, 2) float32
    conics: np.ndarray    # (N, 3) float32
    opacities: np.ndarray  # (N,) float32
    rgb: np.ndarray       # (N, 3) float32
    depth: np.ndarray     # (N,) float32
    cov: np.ndarray       # (N, 3) float64 (xx, xy, yy), the covariance the conic came from
    width: int
    height: int

    @property
    def n(self) -> int:
        return int(self.means2d.shape[0])


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def splats2d(n: int = 1000, width: int = 128, height: int = 128, seed: int = 1,
             log_s_mean: float = math.log(3.0), log_s_sd: float = 0.5) -> Splats2D:
    """2D workload: means uniform over the image, covariance R(theta) diag(s^2) R(theta)^T with
    theta ~ U[0, pi) and log s ~ N(ln 3 px, 0.5), opacity = sigmoid(N(0,1)), rgb ~ U[0,1]^3,
    depth ~ U[0.5, 10]. The conic handed to both sides is fp32 of the fp64 inverse."""
    g = rng(seed)
    means = g.uniform(0.0, 1.0, size=(n, 2)) * np.array([width, height], dtype=np.float64)
    theta = g.uniform(0.0, math.pi, size=n)
    s = np.exp(g.normal(log_s_mean, log_s_sd, size=(n, 2)))
    opac = _sigmoid(g.normal(0.0, 1.0, size=n))
    rgb = g.uniform(0.0, 1.0, size=(n, 3))
    depth = g.uniform(0.5, 10.0, size=n)
    ct, st = np.cos(theta), np.sin(theta)
    s1, s2 = s[:, 0] ** 2, s[:, 1] ** 2
    cxx = ct * ct * s1 + st * st * s2
    cxy = ct * st * (s1 - s2)
    cyy = st * st * s1 + ct * ct * s2
    det = cxx * cyy - cxy * cxy
    conic = np.stack([cyy / det, -cxy / det, cxx / det], axis=1)
    return Splats2D(
        means2d=means.astype(np.float32), conics=conic.astype(np.float32),
        opacities=opac.astype(np.float32), rgb=rgb.astype(np.float32),
        depth=depth.astype(np.float32), cov=np.stack([cxx, cxy, cyy], 1),
        width=width, height=height)


def scene3d(n: int, seed: int, sh_degree: int = 3, n_clusters: int = 64,
            cluster_ball: float = 1.5, cluster_sigma: float = 0.3, shell_frac: float = 0.1,
            shell_radius: float = 5.0, log_scale_mean: float = -4.0,
            log_scale_sd: float = 0.7) -> Scene:
    """Clustered 3D scene: (1 - shell_frac) of the Gaussians in ``n_clusters`` isotropic
    clusters (sigma 0.3) whose centres are uniform in a ball of radius 1.5, the rest uniform
    on a sphere of radius 5; log-scale ~ N(-4, 0.7) per axis; quaternions uniform on S^3
    (normalised 4D normals); opacity = sigmoid(N(0,1)); SH DC ~ U[0,1], higher orders
    N(0, 0.05)."""
    g = rng(seed)
    n_shell = int(round(shell_frac * n))
    n_cl = n - n_shell
    d = g.normal(size=(n_clusters, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    centres = d * (cluster_ball * g.uniform(size=(n_clusters, 1)) ** (1.0 / 3.0))
    assign = g.integers(0, n_clusters, size=n_cl)
    pc = centres[assign] + g.normal(0.0, cluster_sigma, size=(n_cl, 3))
    ds = g.normal(size=(n_shell, 3))
    ds /= np.maximum(np.linalg.norm(ds, axis=1, keepdims=True), 1e-12)
    ps = ds * shell_radius
    means = np.concatenate([pc, ps], axis=0)
    perm = g.permutation(n)
    means = means[perm]
    scales = np.exp(g.normal(log_scale_mean, log_scale_sd, size=(n, 3)))
    q = g.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    opac = _sigmoid(g.normal(0.0, 1.0, size=n))
    K = (sh_degree + 1) ** 2
    sh = np.empty((n, K, 3))
    sh[:, 0, :] = g.uniform(0.0, 1.0, size=(n, 3))
    if K > 1:
        sh[:, 1:, :] = g.normal(0.0, 0.05, size=(n, K - 1, 3))
    return Scene(means3d=means.astype(np.float32), scales=scales.astype(np.float32),
                 quats=q.astype(np.float32), opacities=opac.astype(np.float32),
                 sh=sh.astype(np.float32), sh_degree=sh_degree)


def _lookat(campos: np.ndarray, target: np.ndarray, down: np.ndarray) -> np.ndarray:
    z = target - campos
    z = z / np.linalg.norm(z)
    y = down - np.dot(down, z) * z
    y = y / np.linalg.norm(y)
    x = np.cross(y, z)
    R = np.stack([x, y, z], axis=0)
    t = -R @ campos
    return np.concatenate([R, t[:, None]], axis=1).astype(np.float32)


def camera_front(width: int, height: int, fx: float, distance: float = 4.0,
                 znear: float = 0.2) -> Camera:
    """Camera at (0, 0, -distance) looking at the origin along +z, world y pointing down in the
    image, principal point at the image centre."""
    vm = _lookat(np.array([0.0, 0.0, -distance]), np.zeros(3), np.array([0.0, 1.0, 0.0]))
    return Camera(viewmat=vm, fx=float(fx), fy=float(fx), cx=width / 2.0, cy=height / 2.0,
                  width=width, height=height, znear=znear)


def camera_ring(k: int, count: int = 8, radius: float = 4.0, width: int = 1280,
                height: int = 720, fx: float = 1125.0, znear: float = 0.2) -> Camera:
    """Camera k of ``count`` on a ring of the given radius in the xz-plane (angle 2 pi k / count,
    k = 0 at (0, 0, -radius)), looking at the origin."""
    phi = 2.0 * math.pi * k / count
    pos = np.array([radius * math.sin(phi), 0.0, -radius * math.cos(phi)])
    vm = _lookat(pos, np.zeros(3), np.array([0.0, 1.0, 0.0]))
    return Camera(viewmat=vm, fx=float(fx), fy=float(fx), cx=width / 2.0, cy=height / 2.0,
                  width=width, height=height, znear=znear)


def image_grad(width: int, height: int, seed: int) -> np.ndarray:
    """Stochastic image gradient dL/dC ~ U[-1, 1], planar [3, H, W] float32 (the paper's
    backward-timing protocol, Sec. 4)."""
    return rng(seed).uniform(-1.0, 1.0, size=(3, height, width)).astype(np.float32)


def target_image(width: int, height: int, seed: int) -> np.ndarray:
    return rng(seed).uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)


def sorted_key_case(n: int, seed: int, tie_levels: int = 0) -> np.ndarray:
    """uint32 keys for sort tests. With ``tie_levels`` > 0 the keys take only that many distinct
    values, so stability (ties kept in index order) is exercised; a few keys are 0xFFFFFFFF."""
    g = rng(seed)
    if tie_levels > 0:
        k = g.integers(0, tie_levels, size=n).astype(np.uint64) * np.uint64(2654435761)
        k = (k % np.uint64(0xFFFFFFF0)).astype(np.uint32)
    else:
        k = g.integers(0, 2 ** 32 - 1, size=n, dtype=np.uint64).astype(np.uint32)
    sentinel = g.uniform(size=n) < 0.05
    k[sentinel] = np.uint32(0xFFFFFFFF)
    return k


# ---- named workloads -------------------------------------------------------------------

CFG1 = dict(n=1000, width=128, height=128, seed=1, target_seed=11)
CFG2 = dict(n=200_000, width=1024, height=768, fx=900.0, seed=2, grad_seed=102)
CFG3 = dict(n=1_000_000, width=1600, height=1064, fx=1406.25, seed=3, grad_seed=103)
CFG4 = dict(n_hidden=500_000, n_train=500_000, seed_hidden=40, seed_train=41, fd_seed=42,
            width=1280, height=720, fx=1125.0, cameras=8, steps=300, lr=1e-3)
CFG5_RESOLUTIONS = [(640, 480), (800, 600), (1024, 768), (1280, 720), (1600, 900), (1920, 1080)]


def cfg_camera(cfg: dict) -> Camera:
    return camera_front(cfg["width"], cfg["height"], cfg["fx"])


def serving_scenes(count: int = 16, n_min: float = 5e4, ratio: float = 60.0) -> list:
    """Scene sizes for the serving mix: N_j = round(n_min * ratio^(j / (count-1))), seeds 500+j
    (50k ... 3M, log-spaced)."""
    return [(500 + j, int(round(n_min * ratio ** (j / (count - 1))))) for j in range(count)]


def serving_requests(count: int, rate: float, seed: int = 550, n_scenes: int = 16,
                     frac_fwd: float = 0.7) -> list:
    """Poisson arrivals at ``rate`` per second: (arrival_s, scene_index, (W, H), fwd_only)."""
    g = rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, size=count))
    sc = g.integers(0, n_scenes, size=count)
    res = g.integers(0, len(CFG5_RESOLUTIONS), size=count)
    fwd = g.uniform(size=count) < frac_fwd
    return [(float(t[i]), int(sc[i]), CFG5_RESOLUTIONS[int(res[i])], bool(fwd[i]))
            for i in range(count)]
