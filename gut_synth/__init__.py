"""Seeded synthetic inputs for the 3DGUT rasterizer hot path.

This module only draws random numbers and lays out arrays: particle sets
(means, scales, quaternions, opacities, spherical-harmonic coefficients) and
camera descriptions (intrinsics and world-to-camera poses).  It holds none of
the method's arithmetic (no projection, no unscented transform, no
compositing), so both the FP64 CPU oracle and the HIP path can consume the same
inputs without sharing any code of the method.

The workloads stand in for the paper's trained scenes (MipNeRF360, Tanks &
Temples, ScanNet++ fisheye and Waymo rolling-shutter captures, which are not
available): clustered anisotropic Gaussians plus a distant background shell,
viewed through pinhole, OpenCV-fisheye and rolling-shutter cameras at the
resolutions the paper's datasets use.

Seeds: scene ``1000 + c``, camera ``2000 + c``, perturbation or request
``3000 + c`` for workload ``c``.

A camera is a plain dict:
  model    'pinhole' | 'fisheye'   (OpenCV fisheye, k1..k4)
  shutter  'global' | 'rolling'    (rolling: rows exposed top to bottom)
  width, height, fx, fy, cx, cy, k (4 floats)
  R0, t0   world->camera rotation (3x3) and translation at exposure start
  R1, t1   the same at exposure end (equal to R0, t0 for a global shutter)
All pose values are float64; x_cam = R @ x_world + t, OpenCV axes
(+x right, +y down, +z forward).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Real spherical-harmonic band-0 constant 1/(2 sqrt(pi)); used only to place the
# generated DC colour at the requested value (colour = 1/2 + SH_C0 * beta_00).
SH_C0 = 0.5 / math.sqrt(math.pi)


@dataclass
class Scene:
    """A particle set. Activated parameters (what the kernels take) plus the
    raw parameters they came from (what an optimizer would own)."""
    means: np.ndarray       # [n,3] float32
    scales: np.ndarray      # [n,3] float32, > 0     (= exp(log_scales))
    quats: np.ndarray       # [n,4] float32, (w,x,y,z), not normalised
    opacities: np.ndarray   # [n]   float32, (0,1)   (= sigmoid(logit_opacities))
    sh: np.ndarray          # [n,K,3] float32, K=(deg+1)^2
    sh_degree: int
    log_scales: np.ndarray  # [n,3] float32
    logit_opacities: np.ndarray  # [n] float32

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(self.means[idx].copy(), self.scales[idx].copy(),
                     self.quats[idx].copy(), self.opacities[idx].copy(),
                     self.sh[idx].copy(), self.sh_degree,
                     self.log_scales[idx].copy(), self.logit_opacities[idx].copy())


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def scene_from_raw(means, log_scales, quats, logit_opacities, sh, sh_degree) -> Scene:
    means = np.ascontiguousarray(means, np.float32)
    log_scales = np.ascontiguousarray(log_scales, np.float32)
    logit_opacities = np.ascontiguousarray(logit_opacities, np.float32)
    return Scene(means=means,
                 scales=np.exp(log_scales.astype(np.float64)).astype(np.float32),
                 quats=np.ascontiguousarray(quats, np.float32),
                 opacities=_sigmoid(logit_opacities.astype(np.float64)).astype(np.float32),
                 sh=np.ascontiguousarray(sh, np.float32), sh_degree=int(sh_degree),
                 log_scales=log_scales, logit_opacities=logit_opacities)


def _sh_coeffs(rng, n, degree, dc_lo=0.0, dc_hi=1.0, high_std=0.05):
    k = (degree + 1) ** 2
    sh = np.zeros((n, k, 3), np.float64)
    dc = rng.uniform(dc_lo, dc_hi, size=(n, 3))
    sh[:, 0, :] = (dc - 0.5) / SH_C0
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, high_std, size=(n, k - 1, 3))
    return sh.astype(np.float32)


def _random_quats(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _random_rotations(rng, n):
    """Uniform random rotation matrices (from normalised Gaussian quaternions)."""
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1),
    ], 1)


# ----------------------------------------------------------------------------
# Scenes
# ----------------------------------------------------------------------------

def uniform_scene(n: int, seed: int, degree: int = 0, extent: float = 1.0,
                  log_scale_mean: float = -3.5, log_scale_std: float = 0.5,
                  high_std: float = 0.05) -> Scene:
    """Means U[-extent, extent]^3, log-scales N(mean, std) per axis, uniform
    random unit quaternions, opacity sigmoid(N(0,1)), DC colour U[0,1]^3."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-extent, extent, size=(n, 3))
    log_s = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = _random_quats(rng, n)
    logit = rng.normal(0.0, 1.0, size=n)
    sh = _sh_coeffs(rng, n, degree, high_std=high_std)
    return scene_from_raw(means, log_s, quats, logit, sh, degree)


def clustered_scene(n: int, seed: int, degree: int = 3, n_clusters: int = 200,
                    sphere_frac: float = 0.2, sphere_radius: float = 20.0,
                    center_extent: float = 5.0, cluster_std: float = 0.3,
                    log_scale_mean: float = -4.0, log_scale_std: float = 0.7) -> Scene:
    """(1 - sphere_frac) of the particles in ``n_clusters`` anisotropic Gaussian
    clusters (centres U[-5,5]^3, shape R_k diag(0.3 a_k), a_k ~ U[0.5,1.5]^3),
    the rest on a background sphere of radius 20; log-scales N(-4, 0.7);
    SH degree 3 with DC U[0,1] and higher bands N(0, 0.05)."""
    rng = np.random.default_rng(seed)
    n_sphere = int(round(n * sphere_frac))
    n_clu = n - n_sphere
    per = np.full(n_clusters, n_clu // n_clusters)
    per[: n_clu - per.sum()] += 1
    centers = rng.uniform(-center_extent, center_extent, size=(n_clusters, 3))
    rots = _random_rotations(rng, n_clusters)
    axes = cluster_std * rng.uniform(0.5, 1.5, size=(n_clusters, 3))
    owner = np.repeat(np.arange(n_clusters), per)
    z = rng.normal(size=(n_clu, 3)) * axes[owner]
    clu = centers[owner] + np.einsum("nij,nj->ni", rots[owner], z)
    sph = rng.normal(size=(n_sphere, 3))
    sph = sphere_radius * sph / np.linalg.norm(sph, axis=1, keepdims=True)
    means = np.concatenate([clu, sph], 0)
    log_s = rng.normal(log_scale_mean, log_scale_std, size=(n, 3))
    quats = _random_quats(rng, n)
    logit = rng.normal(0.0, 1.0, size=n)
    sh = _sh_coeffs(rng, n, degree)
    return scene_from_raw(means, log_s, quats, logit, sh, degree)


def perturb_raw(scene: Scene, seed: int, std: float = 0.01) -> Scene:
    """Add N(0, std) to every raw parameter (means, log-scales, quaternions,
    logit opacities, SH)."""
    rng = np.random.default_rng(seed)
    f = lambda a: (a.astype(np.float64) + rng.normal(0.0, std, size=a.shape)).astype(np.float32)
    return scene_from_raw(f(scene.means), f(scene.log_scales), f(scene.quats),
                          f(scene.logit_opacities), f(scene.sh), scene.sh_degree)


# ----------------------------------------------------------------------------
# Cameras
# ----------------------------------------------------------------------------

def look_at(eye, target=(0.0, 0.0, 0.0), down=(0.0, 1.0, 0.0)):
    """World->camera (R, t) for a camera at ``eye`` looking at ``target`` with
    OpenCV axes: +z towards the target, +y along the projection of ``down``."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    x = np.cross(np.asarray(down, np.float64), z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z], 0)
    t = -R @ eye
    return R, t


def _axis_angle(axis, angle):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


def camera(model, width, height, fx, fy=None, cx=None, cy=None, k=(0, 0, 0, 0),
           R0=None, t0=None, R1=None, t1=None, shutter="global"):
    fy = fx if fy is None else fy
    cx = width / 2.0 if cx is None else cx
    cy = height / 2.0 if cy is None else cy
    R0 = np.eye(3) if R0 is None else np.asarray(R0, np.float64)
    t0 = np.zeros(3) if t0 is None else np.asarray(t0, np.float64)
    R1 = R0.copy() if R1 is None else np.asarray(R1, np.float64)
    t1 = t0.copy() if t1 is None else np.asarray(t1, np.float64)
    return dict(model=model, shutter=shutter, width=int(width), height=int(height),
                fx=float(fx), fy=float(fy), cx=float(cx), cy=float(cy),
                k=[float(v) for v in k], R0=R0, t0=t0, R1=R1, t1=t1)


def pinhole_focal(width, hfov_deg=60.0):
    """Focal length giving a horizontal field of view of ``hfov_deg``."""
    return width / (2.0 * math.tan(math.radians(hfov_deg) / 2.0))


def fisheye_focal(width, fov_deg=180.0):
    """Equidistant focal length mapping half the width to half the FOV."""
    return (width / 2.0) / math.radians(fov_deg / 2.0)


def with_motion(cam, pan_rad, shift):
    """Rolling-shutter copy of ``cam``: between the first and last row the
    camera pans by ``pan_rad`` about its own y axis and moves ``shift`` units
    along its own x axis."""
    R0, t0 = cam["R0"], cam["t0"]
    Q0 = R0.T                        # camera->world
    c0 = -R0.T @ t0
    Q1 = Q0 @ _axis_angle([0.0, 1.0, 0.0], pan_rad)
    c1 = c0 + shift * Q0[:, 0]
    R1 = Q1.T
    t1 = -R1 @ c1
    out = dict(cam)
    out.update(R1=R1, t1=t1, shutter="rolling")
    return out


def random_fisheye_k(rng, lo=-0.05, hi=0.05):
    return [float(v) for v in rng.uniform(lo, hi, size=4)]


def random_eye(rng, radius=8.0, max_abs_y=0.99):
    while True:
        v = rng.normal(size=3)
        v = v / np.linalg.norm(v)
        if abs(v[1]) <= max_abs_y:
            return radius * v


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------

def config1(n=1000, width=128, height=128):
    """1,000 Gaussians in U[-1,1]^3, SH degree 0, pinhole 128x128 at (0,0,-3)
    looking at the origin with fx = fy = 150."""
    scene = uniform_scene(n, seed=1001, degree=0)
    R, t = look_at((0.0, 0.0, -3.0))
    cam = camera("pinhole", width, height, 150.0 * width / 128.0,
                 R0=R, t0=t)
    return scene, [cam]


def config2_scene(n=1_000_000):
    return clustered_scene(n, seed=1002)


def config2_cameras(width=1920, height=1080):
    """Pinhole (60 deg horizontal FOV) and 180-deg OpenCV fisheye views from
    (0,0,-8) looking at the origin."""
    rng = np.random.default_rng(2002)
    R, t = look_at((0.0, 0.0, -8.0))
    pin = camera("pinhole", width, height, pinhole_focal(width), R0=R, t0=t)
    fish = camera("fisheye", width, height, fisheye_focal(width),
                  k=random_fisheye_k(rng), R0=R, t0=t)
    return [pin, fish]


def config3_scene(n=3_000_000):
    return clustered_scene(n, seed=1003)


def config3_camera(width=1600, height=1200):
    """180-deg fisheye 1600x1200 with a rolling shutter: 0.1 rad pan about the
    camera y axis and 0.3 units along camera x between the first and last
    row."""
    rng = np.random.default_rng(2003)
    R, t = look_at((0.0, 0.0, -8.0))
    cam = camera("fisheye", width, height, fisheye_focal(width),
                 k=random_fisheye_k(rng), R0=R, t0=t)
    return with_motion(cam, 0.1, 0.3)


def config4_gradcheck(kind="pinhole", n=64, log_scale_mean=-3.5):
    """64 Gaussians (the config-1 recipe with SH degree 3) seen by a 32x32
    camera at (0,0,-3); ``kind`` in {'pinhole', 'fisheye', 'rolling'}.
    ``log_scale_mean`` above the recipe's -3.5 gives larger, more overlapping
    particles for a denser gradient check."""
    scene = uniform_scene(n, seed=1004, degree=3, log_scale_mean=log_scale_mean)
    R, t = look_at((0.0, 0.0, -3.0))
    if kind == "pinhole":
        cam = camera("pinhole", 32, 32, 37.5, R0=R, t0=t)
    else:
        rng = np.random.default_rng(2004)
        cam = camera("fisheye", 32, 32, fisheye_focal(32, 120.0),
                     k=random_fisheye_k(rng), R0=R, t0=t)
        if kind == "rolling":
            cam = with_motion(cam, 0.1, 0.3)
    return scene, cam


def config5_requests(n_requests, seed=3005, max_cams=8):
    """Serving trace: each request holds U{1..8} cameras, half pinhole at a
    resolution drawn from 640x480 .. 3840x2160 (60 deg FOV), half 180-deg
    rolling-shutter fisheye 1600x1200 with the config-3 intrinsics and motion;
    eyes on a sphere of radius 8 facing the origin."""
    rng = np.random.default_rng(seed)
    sizes = [(640, 480), (1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)]
    fish_k = config3_camera()["k"]
    reqs = []
    for _ in range(n_requests):
        cams = []
        for _ in range(int(rng.integers(1, max_cams + 1))):
            R, t = look_at(random_eye(rng))
            if rng.random() < 0.5:
                w, h = sizes[int(rng.integers(0, len(sizes)))]
                cams.append(camera("pinhole", w, h, pinhole_focal(w), R0=R, t0=t))
            else:
                c = camera("fisheye", 1600, 1200, fisheye_focal(1600), k=fish_k,
                           R0=R, t0=t)
                cams.append(with_motion(c, 0.1, 0.3))
        reqs.append(cams)
    return reqs


def poisson_arrivals(n, rate_per_s, seed):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
