"""Seeded synthetic inputs: scenes, cameras and settings.

This module only draws random numbers and builds plain containers; it holds
none of the rendering method's arithmetic and is shared by the tests, the
benchmark and the CPU oracle harness.

Scene layout (structure of arrays, float32, contiguous):
    means          [3][N]
    log_scales     [3][N]
    quats          [4][N]   (w, x, y, z), not necessarily unit length
    opacity_logits [N]
    sh             [(D+1)^2][3][N]
    v_train        [N] or None   per-Gaussian training sampling frequency (pixels per unit)

Camera: world->view rigid 4x4 (row-major, +x right, +y down, +z forward),
pinhole intrinsics in pixels, image size, near-plane depth and background.
The workload shapes follow the paper's evaluation setting (Sec. 4): trained
scenes of ~0.5-3M Gaussians rendered at dataset resolutions; the datasets and
trained models are not available, so seeded synthetic scenes of the same
shape stand in for them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

SH_C0 = 0.28209479177387814  # 1 / (2 sqrt(pi)), used only to encode a base colour


@dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    v_train: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    @property
    def sh_degree(self) -> int:
        nb = self.sh.shape[0]
        d = int(round(math.sqrt(nb))) - 1
        assert (d + 1) ** 2 == nb
        return d

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(
            means=np.ascontiguousarray(self.means[:, idx]),
            log_scales=np.ascontiguousarray(self.log_scales[:, idx]),
            quats=np.ascontiguousarray(self.quats[:, idx]),
            opacity_logits=np.ascontiguousarray(self.opacity_logits[idx]),
            sh=np.ascontiguousarray(self.sh[:, :, idx]),
            v_train=None if self.v_train is None else np.ascontiguousarray(self.v_train[idx]),
        )

    def concat(self, other: "Scene") -> "Scene":
        vt = None
        if self.v_train is not None and other.v_train is not None:
            vt = np.concatenate([self.v_train, other.v_train])
        return Scene(
            means=np.ascontiguousarray(np.concatenate([self.means, other.means], 1)),
            log_scales=np.ascontiguousarray(np.concatenate([self.log_scales, other.log_scales], 1)),
            quats=np.ascontiguousarray(np.concatenate([self.quats, other.quats], 1)),
            opacity_logits=np.ascontiguousarray(np.concatenate([self.opacity_logits, other.opacity_logits])),
            sh=np.ascontiguousarray(np.concatenate([self.sh, other.sh], 2)),
            v_train=vt,
        )


@dataclass
class Camera:
    viewmat: np.ndarray  # (4, 4) float64, world -> view
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    znear: float = 0.01
    bg: tuple = (0.0, 0.0, 0.0)

    @property
    def position(self) -> np.ndarray:
        R = self.viewmat[:3, :3]
        t = self.viewmat[:3, 3]
        return -R.T @ t

    @property
    def tiles(self) -> tuple:
        return ((self.width + 15) // 16, (self.height + 15) // 16)


@dataclass
class Settings:
    filter_k: float = 0.3          # Sec. 4 implementation details
    ray_window: int = 16           # per-ray window K (0 = blend in tile order)
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_min: float = 1e-4
    filter_mode: int = 0           # 0 adaptive (Eq.12), 1 off, 2 volume-normalised (Eq.8)
    tile_cull: bool = True         # 3D per-tile culling (Sec. 3.4); False = rectangle only
    subtile_sort: bool = False     # middle level: exact re-sort per 8x8 sub-tile by its centre-line depth


def look_at(position, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """World->view matrix: +z towards target, +x right, +y down."""
    p = np.asarray(position, np.float64)
    f = np.asarray(target, np.float64) - p
    f /= np.linalg.norm(f)
    u = np.asarray(up, np.float64)
    if abs(np.dot(f, u / np.linalg.norm(u))) > 0.999:
        u = np.array([0.0, 0.0, 1.0])
    right = np.cross(f, u)
    right /= np.linalg.norm(right)
    down = np.cross(f, right)
    V = np.eye(4)
    V[0, :3], V[1, :3], V[2, :3] = right, down, f
    V[:3, 3] = -V[:3, :3] @ p
    return V


def pinhole(position, width, height, fov_x_deg, target=(0.0, 0.0, 0.0), znear=0.01, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera with horizontal field of view fov_x, square pixels, principal point at the centre."""
    fx = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    return Camera(look_at(position, target), fx, fx, width / 2.0, height / 2.0, int(width), int(height), znear, tuple(bg))


def sphere_poses(rng: np.random.Generator, count: int, radius: float) -> np.ndarray:
    d = rng.normal(size=(count, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * radius


def _random_quats(rng, n):
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _base_colour_sh(rng, n, degree, ac_std):
    nb = (degree + 1) ** 2
    sh = np.zeros((nb, 3, n), np.float64)
    if degree > 0:
        sh[1:] = rng.normal(0.0, ac_std, size=(nb - 1, 3, n))
    u = rng.uniform(0.0, 1.0, size=(3, n))
    sh[0] = (u - 0.5) / SH_C0
    return sh


def rig_frequency(means: np.ndarray, rig_radius: float, rig_fx: float) -> np.ndarray:
    """Stand-in for the stored per-Gaussian training sampling frequency (a
    renderer input: pixels per world unit).  A trainer would record it from
    its cameras; here it is drawn from the rig's shape alone: its focal
    length over the smallest distance a camera on the rig sphere can have
    from the mean (the sphere radius minus the mean's distance from the
    centre, at least a twentieth of the radius).  Plain input data: no
    visibility, no camera poses."""
    r = np.linalg.norm(means.astype(np.float64), axis=0)
    d = np.maximum(rig_radius - r, 0.05 * rig_radius)
    return (rig_fx / d).astype(np.float32)


def _focal(width, fov_x_deg):
    return (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)


def _finish(means, log_scales, quats, logits, sh, v_train) -> Scene:
    f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Scene(f32(means), f32(log_scales), f32(quats), f32(logits), f32(sh), None if v_train is None else f32(v_train))


# ----------------------------------------------------------------------------
# Workloads.  Seeds are fixed per workload; every result records them.


def small_scene(n=2000, seed=1001, sh_degree=0, with_v_train=True):
    """2k Gaussians, means U[-1,1]^3, log-scales N(-3,0.5), uniform random
    rotations, logits N(0,1), base colour U[0,1]; camera 128x128, 60 deg,
    distance 3 looking at the origin; training rig of 8 poses at distance 3."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(3, n))
    log_scales = rng.normal(-3.0, 0.5, size=(3, n))
    quats = _random_quats(rng, n)
    logits = rng.normal(0.0, 1.0, size=n)
    sh = _base_colour_sh(rng, n, sh_degree, 0.1)
    sphere_poses(rng, 8, 3.0)  # keeps the draw sequence of the rig
    v_train = rig_frequency(means, 3.0, _focal(128, 60.0)) if with_v_train else None
    cam = pinhole(sphere_poses(rng, 1, 3.0)[0], 128, 128, 60.0)
    return _finish(means, log_scales, quats, logits, sh, v_train), cam


def cluster_scene(n, seed=1002, sh_degree=3, n_clusters=64, box=10.0, log_scale_mu=-4.0, log_scale_sd=0.7,
                  n_rig=32, rig_radius=12.0, rig_w=1920, rig_h=1080, rig_fov=60.0):
    """Mixture of anisotropic clusters inside a 2*box cube.  Cluster centres
    U[-box,box]^3, cluster covariance Rc diag(sigma^2) Rc^T with sigma
    U[0.25,2.5]^3, means rejection-sampled into the box; log-scales
    N(-4,0.7); logits N(0.5,1.5); SH3 coefficients N(0,0.1) with the DC term
    encoding a U[0,1] base colour.  n_rig poses on a sphere of rig_radius
    (the benchmark views); v_train from the rig's radius and focal length."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box, box, size=(n_clusters, 3))
    sig = rng.uniform(0.25, 2.5, size=(n_clusters, 3))
    rots = []
    for _ in range(n_clusters):
        q, _r = np.linalg.qr(rng.normal(size=(3, 3)))
        rots.append(q)
    rots = np.stack(rots)
    means = np.empty((n, 3))
    filled = 0
    while filled < n:
        m = (n - filled) * 2 + 1024
        cid = rng.integers(0, n_clusters, size=m)
        z = rng.normal(size=(m, 3)) * sig[cid]
        pts = centres[cid] + np.einsum("mij,mj->mi", rots[cid], z)
        ok = np.all(np.abs(pts) <= box, axis=1)
        pts = pts[ok][: n - filled]
        means[filled: filled + len(pts)] = pts
        filled += len(pts)
    means = means.T.copy()
    log_scales = rng.normal(log_scale_mu, log_scale_sd, size=(3, n))
    quats = _random_quats(rng, n)
    logits = rng.normal(0.5, 1.5, size=n)
    sh = _base_colour_sh(rng, n, sh_degree, 0.1)
    rig_pos = sphere_poses(rng, n_rig, rig_radius)
    v_train = rig_frequency(means, rig_radius, _focal(rig_w, rig_fov))
    return _finish(means, log_scales, quats, logits, sh, v_train), rig_pos


def headline(n=1_000_000, seed=1002):
    """1M Gaussians of the cluster generator, 1920x1080, 60 deg, SH3; the
    benchmark poses are the 32 rig poses at radius 12."""
    scene, poses = cluster_scene(n, seed=seed)
    cams = [pinhole(p, 1920, 1080, 60.0) for p in poses]
    return scene, cams


def medium(n=500_000, seed=1002):
    scene, poses = cluster_scene(n, seed=seed)
    cams = [pinhole(p, 1920, 1080, 60.0) for p in poses]
    return scene, cams


def ood_scene(n=3_000_000, seed=1003, near_frac=0.1):
    """Out-of-distribution views: cluster generator at 2064x2208, 120 deg;
    near_frac of the Gaussians re-placed within 0.5 of the primary camera with
    view depth U[znear-0.1, znear+0.1] (straddling the near plane and z=0)."""
    scene, poses = cluster_scene(n, seed=seed)
    rng = np.random.default_rng(seed + 100)
    cam = pinhole(poses[0], 2064, 2208, 120.0)
    k = int(n * near_frac)
    idx = rng.choice(n, size=k, replace=False)
    # positions in view space: lateral offsets inside a 0.5 ball
    zv = rng.uniform(cam.znear - 0.1, cam.znear + 0.1, size=k)
    r = 0.5 * np.sqrt(rng.uniform(0, 1, size=k)) * np.sqrt(np.maximum(0.0, 1.0 - (zv / 0.5) ** 2))
    ang = rng.uniform(0, 2 * np.pi, size=k)
    Xv = np.stack([r * np.cos(ang), r * np.sin(ang), zv])
    R = cam.viewmat[:3, :3]
    t = cam.viewmat[:3, 3:4]
    Xw = R.T @ (Xv - t)
    scene.means[:, idx] = Xw.astype(np.float32)
    zoom = []
    rs = 10.0 * math.sqrt(3.0)
    d0 = poses[0] / np.linalg.norm(poses[0])
    for k_ in range(8):
        dist = 2.0 * 32.0 ** (k_ / 7.0) * rs
        zoom.append(pinhole(d0 * dist, 2064, 2208, 120.0))
    return scene, cam, zoom


def fwd_bwd_scene(n=1_000_000, seed=1004):
    scene, poses = cluster_scene(n, seed=seed, n_rig=16, rig_w=1280, rig_h=720, rig_fov=70.0)
    cams = [pinhole(p, 1280, 720, 70.0) for p in poses]
    return scene, cams


def fd_scene(n=64, seed=1005):
    """Tiny scene for finite differences: 64 Gaussians, 32x32, log-scales N(-2,0.3)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(3, n)) * 0.6
    log_scales = rng.normal(-2.0, 0.3, size=(3, n))
    quats = _random_quats(rng, n)
    logits = rng.normal(0.0, 1.0, size=n)
    sh = _base_colour_sh(rng, n, 3, 0.1)
    sphere_poses(rng, 8, 3.0)  # keeps the draw sequence of the rig
    v_train = rig_frequency(means, 3.0, _focal(32, 60.0))
    cam = pinhole(sphere_poses(rng, 1, 3.0)[0], 32, 32, 60.0)
    return _finish(means, log_scales, quats, logits, sh, v_train), cam


def noise_target(height, width, seed=1006):
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)
