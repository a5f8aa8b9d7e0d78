"""Seeded scene and camera generators (NumPy ``default_rng``).

Layouts match the C ABI: structure-of-arrays, float32, primitive index fastest.

  mu      [3][N]   centres
  q       [4][N]   rotation quaternions (w, x, y, z), unit length
  scale   [K][N]   radial basis lengths s_k > 0
  theta   [K][N]   basis polar angles, ascending in [0, 2*pi), every gap < pi
  eta     [N]      L1/L2 blend weight in [0, 1]
  tau     [N]      edge sharpness in [0, 0.99]
  opacity [N]      o in [0.05, 0.99]
  color   [C][N]   RGB (C = 3) or degree-3 SH coefficients (C = 48, row = 3*coef + channel)

Cameras are OpenCV pinholes (x right, y down, z forward) with a world-to-camera
rotation R and translation t, pixel centres at integer + 0.5.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO_PI_F32_BELOW = np.nextafter(np.float32(2 * math.pi), np.float32(0))


@dataclasses.dataclass
class Scene:
    mu: np.ndarray
    q: np.ndarray
    scale: np.ndarray
    theta: np.ndarray
    eta: np.ndarray
    tau: np.ndarray
    opacity: np.ndarray
    color: np.ndarray
    sh_degree: int = -1          # -1: plain RGB colours; 0..3: SH of that degree

    @property
    def n(self) -> int:
        return int(self.mu.shape[1])

    @property
    def K(self) -> int:
        return int(self.scale.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(*(getattr(self, f.name)[..., idx] if f.name != "sh_degree" else self.sh_degree
                       for f in dataclasses.fields(self)))

    def nbytes(self) -> int:
        return sum(getattr(self, f.name).nbytes for f in dataclasses.fields(self) if f.name != "sh_degree")


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray                # (3, 3) float32, world -> camera
    t: np.ndarray                # (3,) float32
    bg: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3, np.float32))

    def position(self) -> np.ndarray:
        return -(self.R.astype(np.float64).T @ self.t.astype(np.float64))


def intrinsics_hfov(width: int, height: int, hfov_deg: float = 60.0):
    """Focal length from a horizontal field of view; principal point at the image centre."""
    f = width / (2.0 * math.tan(math.radians(hfov_deg) / 2.0))
    return np.float32(f), np.float32(f), np.float32(width / 2.0), np.float32(height / 2.0)


def camera_lookat(eye, target, up, width, height, hfov_deg=60.0, bg=(0.0, 0.0, 0.0)) -> Camera:
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    down = -np.asarray(up, np.float64)
    x = np.cross(down, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z]).astype(np.float32)
    t = (-(R.astype(np.float64) @ eye)).astype(np.float32)
    fx, fy, cx, cy = intrinsics_hfov(width, height, hfov_deg)
    return Camera(width, height, fx, fy, cx, cy, R, t, np.asarray(bg, np.float32))


def camera_from_yaw_pitch(eye, yaw, pitch, width, height, hfov_deg=60.0, bg=(0.0, 0.0, 0.0)) -> Camera:
    """Camera at ``eye`` looking along (cos p cos y, cos p sin y, sin p); world up is +z."""
    fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    return camera_lookat(eye, np.asarray(eye, np.float64) + fwd, (0.0, 0.0, 1.0), width, height, hfov_deg, bg)


def draw_quaternions(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def draw_angles(rng, K, n):
    """Sorted uniform angles in [0, 2*pi); rows with any gap (wrap included) >= pi are redrawn."""
    th = np.sort(rng.uniform(0.0, 2 * math.pi, size=(n, K)), axis=1).astype(np.float32)
    th = np.minimum(th, TWO_PI_F32_BELOW)

    def bad_rows(a):
        a64 = a.astype(np.float64)
        gaps = np.diff(np.concatenate([a64, a64[:, :1] + 2 * math.pi], axis=1), axis=1)
        return np.nonzero(gaps.max(axis=1) >= math.pi)[0]

    bad = bad_rows(th)
    while bad.size:
        redo = np.sort(rng.uniform(0.0, 2 * math.pi, size=(bad.size, K)), axis=1).astype(np.float32)
        th[bad] = np.minimum(redo, TWO_PI_F32_BELOW)
        bad = bad[bad_rows(th[bad])]
    return np.ascontiguousarray(th.T)


def _log_uniform(rng, lo, hi, shape):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size=shape)).astype(np.float32)


def _common_params(rng, n, K, s_lo, s_hi):
    q = draw_quaternions(rng, n)
    scale = _log_uniform(rng, s_lo, s_hi, (K, n))
    theta = draw_angles(rng, K, n)
    eta = rng.uniform(0.0, 1.0, n).astype(np.float32)
    tau = rng.uniform(0.0, 0.99, n).astype(np.float32)
    opacity = rng.uniform(0.05, 0.99, n).astype(np.float32)
    return q, scale, theta, eta, tau, opacity


def _sh_colors(rng, n, degree=3):
    nc = (degree + 1) ** 2
    col = rng.normal(0.0, 0.05, size=(nc, 3, n))
    col[0] = rng.uniform(0.0, 1.0, size=(3, n))
    return col.reshape(nc * 3, n).astype(np.float32)


def scene_uniform_box(seed, n, K=8, half=1.0, s_lo=0.02, s_hi=0.3) -> Scene:
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-half, half, size=(3, n)).astype(np.float32)
    q, scale, theta, eta, tau, opacity = _common_params(rng, n, K, s_lo, s_hi)
    color = rng.uniform(0.0, 1.0, size=(3, n)).astype(np.float32)
    return Scene(mu, q, scale, theta, eta, tau, opacity, color, -1)


def scene_sphere_shell(seed, n, K=8, s_lo=0.02, s_hi=0.3, sh_degree=3) -> Scene:
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    r = 1.0 + rng.normal(0.0, 0.05, n)
    mu = (d * r).astype(np.float32)
    q, scale, theta, eta, tau, opacity = _common_params(rng, n, K, s_lo, s_hi)
    color = _sh_colors(rng, n, sh_degree)
    return Scene(mu, q, scale, theta, eta, tau, opacity, color, sh_degree)


def scene_clusters(seed, n, K=8, half=10.0, n_clusters=64, s_lo=0.005, s_hi=0.5, sh_degree=3,
                   cluster_scale=1.0) -> Scene:
    """Mixture of anisotropic 3D Gaussian clusters in the box [-half, half]^3 (equal weights)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-half, half, size=(n_clusters, 3))
    A = np.empty((n_clusters, 3, 3))
    for c in range(n_clusters):
        g, r = np.linalg.qr(rng.standard_normal((3, 3)))
        rot = g * np.sign(np.diag(r))[None, :]
        A[c] = rot @ np.diag(rng.uniform(0.3, 2.0, 3) * cluster_scale)
    which = rng.integers(0, n_clusters, n)
    z = rng.standard_normal((n, 3))
    pts = centres[which] + np.einsum("nij,nj->ni", A[which], z)
    mu = np.clip(pts, -half, half).T.astype(np.float32)
    q, scale, theta, eta, tau, opacity = _common_params(rng, n, K, s_lo, s_hi)
    color = _sh_colors(rng, n, sh_degree)
    return Scene(np.ascontiguousarray(mu), q, scale, theta, eta, tau, opacity, color, sh_degree)


def random_target(seed, height, width):
    rng = np.random.default_rng(seed + 1000)
    return rng.uniform(0.0, 1.0, size=(3, height, width)).astype(np.float32)


# ---------------------------------------------------------------------------------------------
# The five workloads (sizes and laws as stated for the synthetic benchmarks)

def config_c1():
    """64x64, 256 DRKs (K=8), centres in [-1,1]^3, RGB, camera at z=-4 looking at the origin."""
    scene = scene_uniform_box(0, 256, K=8)
    fx, fy, cx, cy = intrinsics_hfov(64, 64, 60.0)
    cam = Camera(64, 64, fx, fy, cx, cy, np.eye(3, dtype=np.float32),
                 np.array([0.0, 0.0, 4.0], np.float32), np.zeros(3, np.float32))
    return scene, cam


def config_c2(n=100_000, width=800, height=800):
    """100k DRKs on a unit-sphere shell, SH3, camera on a radius-4 orbit looking at the origin."""
    scene = scene_sphere_shell(1, n, K=8)
    rng = np.random.default_rng(101)
    az = rng.uniform(0.0, 2 * math.pi)
    el = math.radians(rng.uniform(-30.0, 30.0))
    eye = 4.0 * np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    cam = camera_lookat(eye, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0), width, height, 60.0)
    return scene, cam


def c3_camera_path(seed, n_frames, width, height, half=10.0):
    """Smooth seeded path inside the central 80% of the box: 0.05 units/frame along the view
    direction, yaw +1 degree per frame, pitch slowly varying in [-30, 30] degrees."""
    rng = np.random.default_rng(seed)
    lim = 0.8 * half
    pos = rng.uniform(-0.5 * lim, 0.5 * lim, 3)
    yaw0 = rng.uniform(0.0, 2 * math.pi)
    p0 = rng.uniform(-25.0, 25.0)
    ph = rng.uniform(0.0, 2 * math.pi)
    cams = []
    for i in range(n_frames):
        yaw = yaw0 + math.radians(i)
        pitch = math.radians(float(np.clip(p0 + 5.0 * math.sin(ph + 2 * math.pi * i / 100.0), -30.0, 30.0)))
        cams.append(camera_from_yaw_pitch(pos.copy(), yaw, pitch, width, height, 60.0))
        fwd = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
        pos = np.clip(pos + 0.05 * fwd, -lim, lim)
    return cams


def config_c3(n=1_000_000, width=1920, height=1080, n_frames=100):
    """1M DRKs in 64 anisotropic clusters of a 20-unit box, SH3; camera path inside the box."""
    scene = scene_clusters(2, n, K=8, half=10.0)
    cams = c3_camera_path(202, n_frames, width, height, half=10.0)
    return scene, cams


def config_c4_scenes(n_scenes=16, lo=50_000, hi=1_000_000):
    sizes = np.round(np.geomspace(lo, hi, n_scenes)).astype(int)
    return [scene_clusters(3 * 1000 + i, int(s), K=8, half=10.0) for i, s in enumerate(sizes)]


def config_c5(n=3_000_000, width=1920, height=1080, n_views=8):
    """3M DRKs, K=16, SH3, clusters in a 40-unit box; 8 views of the same scene."""
    scene = scene_clusters(4, n, K=16, half=20.0, cluster_scale=2.0)
    cams = c3_camera_path(404, 8 * n_views, width, height, half=20.0)[::8]
    return scene, cams
