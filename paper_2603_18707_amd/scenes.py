"""Seeded synthetic scenes and cameras.

This module only draws inputs: it holds none of the rendering arithmetic, so
the GPU path and the reference can both take their inputs from it. The paper
measures on trained Mip-NeRF 360, Tanks and Temples and Deep Blending scenes
(1.05M-4.9M splats, Table 5); those are not available, and these generators
stand in for them with the splat counts, scale and opacity distributions and
resolutions of the workloads below.

Scenes are returned in activated form (the form the C ABI takes): scales are
standard deviations (exp of log-scales), quaternions (w, x, y, z) are
normalised, opacities are sigmoid(logit), and colours are real spherical
harmonic coefficients [n, (d+1)^2, 3].
"""
import math
from dataclasses import dataclass, replace

import numpy as np


@dataclass
class Scene:
    means3d: np.ndarray   # [n, 3] float32
    scales: np.ndarray    # [n, 3] float32, standard deviations
    quats: np.ndarray     # [n, 4] float32, (w, x, y, z)
    opacities: np.ndarray  # [n] float32 in [0, 1]
    sh: np.ndarray        # [n, (d+1)^2, 3] float32
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means3d.shape[0])

    def subset(self, idx) -> "Scene":
        return Scene(self.means3d[idx].copy(), self.scales[idx].copy(), self.quats[idx].copy(),
                     self.opacities[idx].copy(), self.sh[idx].copy(), self.sh_degree)


@dataclass
class Camera:
    viewmat: np.ndarray  # [4, 4] float32 world -> camera (x right, y down, z forward), row-major
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


def _f32(x: float) -> float:
    return float(np.float32(x))


def pinhole(width: int, height: int, fov_x_deg: float, viewmat=None) -> Camera:
    """Pinhole camera with horizontal field of view fov_x and the principal
    point at the image centre; every intrinsic is a float32 value."""
    f = (width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)
    vm = np.eye(4, dtype=np.float32) if viewmat is None else np.asarray(viewmat, np.float32)
    return Camera(vm, _f32(f), _f32(f), _f32(width / 2.0), _f32(height / 2.0), int(width), int(height))


def look_at(eye, target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0)) -> np.ndarray:
    """World -> camera matrix of a camera at ``eye`` looking at ``target``,
    camera axes x right, y down, z forward."""
    eye, target, up = (np.asarray(v, np.float64) for v in (eye, target, up))
    z = target - eye
    z /= np.linalg.norm(z)
    down = -up
    x = np.cross(down, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    vm = np.eye(4)
    vm[:3, :3] = R
    vm[:3, 3] = -R @ eye
    return vm.astype(np.float32)


def orbit_camera(width, height, azimuth, elevation=0.0, radius=30.0, fov_x_deg=60.0) -> Camera:
    """Camera on a sphere of ``radius`` around the origin looking at it
    (azimuth 0, elevation 0 is the point (0, 0, -radius))."""
    ce = math.cos(elevation)
    eye = (radius * math.sin(azimuth) * ce, radius * math.sin(elevation), -radius * math.cos(azimuth) * ce)
    return pinhole(width, height, fov_x_deg, look_at(eye))


def _random_quats(rng, n) -> np.ndarray:
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def tiny_scene(n: int = 1000, seed: int = 1, sh_degree: int = 0, sh_sigma: float = 0.3):
    """Tiny scene: means uniform in [-1,1]^3 placed 4 units in front of an
    identity camera, log-scales N(-3, 0.5), random unit quaternions, opacity
    sigmoid(N(0, 1.5)). With sh_degree 0 the DC coefficient is drawn so that the
    colour is uniform in [0, 1] (DC uniform on [-sqrt(pi), sqrt(pi)]); higher
    degrees draw every coefficient from N(0, sh_sigma)."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(-1.0, 1.0, size=(n, 3)) + np.array([0.0, 0.0, 4.0])
    scales = np.exp(rng.normal(-3.0, 0.5, size=(n, 3)))
    quats = _random_quats(rng, n)
    opac = _sigmoid(rng.normal(0.0, 1.5, size=n))
    nb = (sh_degree + 1) ** 2
    if sh_degree == 0:
        sh = rng.uniform(-math.sqrt(math.pi), math.sqrt(math.pi), size=(n, 1, 3))
    else:
        sh = rng.normal(0.0, sh_sigma, size=(n, nb, 3))
    return Scene(means.astype(np.float32), scales.astype(np.float32), quats, opac.astype(np.float32),
                 sh.astype(np.float32), sh_degree)


def tiny_camera(width: int = 128, height: int = 128) -> Camera:
    return pinhole(width, height, 60.0)


def cluster_scene(n: int, seed: int, sh_degree: int = 3, logscale=("normal", -4.5, 1.0),
                  opacity_logit=(0.0, 2.0), n_clusters: int = 64, box: float = 10.0,
                  logscale_cap: float = math.log(5.0)):
    """Scene-scale generator: means from a mixture of ``n_clusters`` anisotropic
    Gaussian clusters with centres uniform in [-box, box]^3 and per-cluster
    covariance R diag(U(0.3, 3))^2 R^T, clipped to the box; log-scales from
    N(loc, scale) or a Student-t ("t", nu, loc, scale), capped at
    ``logscale_cap``; random unit quaternions; opacity sigmoid(N(mu, sigma));
    SH coefficients N(0, 0.3)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-box, box, size=(n_clusters, 3))
    rots = []
    for _ in range(n_clusters):
        q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        rots.append(q)
    sds = rng.uniform(0.3, 3.0, size=(n_clusters, 3))
    lab = rng.integers(0, n_clusters, size=n)
    z = rng.normal(size=(n, 3)) * sds[lab]
    R = np.stack(rots)[lab]
    means = centres[lab] + np.einsum("nij,nj->ni", R, z)
    means = np.clip(means, -box, box)
    if logscale[0] == "normal":
        ls = rng.normal(logscale[1], logscale[2], size=(n, 3))
    else:
        _, nu, loc, sc = logscale
        ls = loc + sc * rng.standard_t(nu, size=(n, 3))
    ls = np.minimum(ls, logscale_cap)
    scales = np.exp(ls)
    quats = _random_quats(rng, n)
    opac = _sigmoid(rng.normal(opacity_logit[0], opacity_logit[1], size=n))
    nb = (sh_degree + 1) ** 2
    sh = rng.normal(0.0, 0.3, size=(n, nb, 3))
    return Scene(means.astype(np.float32), scales.astype(np.float32), quats, opac.astype(np.float32),
                 sh.astype(np.float32), sh_degree)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

def workload_tiny():
    """1,000 splats, SH degree 0, one 128x128 camera (fov 60 deg)."""
    return tiny_scene(1000, seed=1), tiny_camera()


def workload_scene(n: int = 1_000_000, seed: int = 2, width: int = 1920, height: int = 1080):
    """1M splats, SH degree 3, one 1920x1080 camera at (0, 0, -30) looking at
    the origin with a 60 deg horizontal field of view."""
    return cluster_scene(n, seed), orbit_camera(width, height, 0.0)


def workload_heavy(n: int = 4_000_000, seed: int = 3, width: int = 1920, height: int = 1080, views: int = 8):
    """4M splats with Student-t(3, -4.5, 0.8) log-scales (capped at ln 5) and
    opacity logits N(1, 2.5); 8 cameras on an orbit of radius 30, 45 deg apart."""
    scene = cluster_scene(n, seed, logscale=("t", 3.0, -4.5, 0.8), opacity_logit=(1.0, 2.5))
    cams = [orbit_camera(width, height, 2.0 * math.pi * k / views) for k in range(views)]
    return scene, cams


BATCH_SCENE_SIZES = (100_000, 250_000, 500_000, 1_000_000, 1_500_000, 2_000_000)
BATCH_RESOLUTIONS = ((640, 360), (1280, 720), (1600, 900), (1920, 1080))


def workload_batched(sizes=BATCH_SCENE_SIZES, views_per_scene: int = 16, seed: int = 46):
    """Six scenes of the scene-scale generator (seeds 40-45) with 16 cameras
    each on the radius-30 orbit: azimuth U(0, 2 pi), elevation U(-15, 15) deg,
    resolution uniform over 640x360, 1280x720, 1600x900, 1920x1080."""
    scenes = [cluster_scene(n, 40 + k) for k, n in enumerate(sizes)]
    rng = np.random.default_rng(seed)
    views = []  # (scene index, camera)
    for s in range(len(scenes)):
        for _ in range(views_per_scene):
            az = rng.uniform(0.0, 2.0 * math.pi)
            el = math.radians(rng.uniform(-15.0, 15.0))
            w, h = BATCH_RESOLUTIONS[int(rng.integers(0, len(BATCH_RESOLUTIONS)))]
            views.append((s, orbit_camera(w, h, az, el)))
    return scenes, views


def workload_train(n: int = 500_000, seed: int = 5, width: int = 1280, height: int = 720, views: int = 4):
    """500k splats, 4 orbit views at 1280x720, and targets rendered from the
    same scene with means + N(0, 0.01) and opacity logits + N(0, 0.2)."""
    scene = cluster_scene(n, seed)
    cams = [orbit_camera(width, height, 2.0 * math.pi * k / views) for k in range(views)]
    rng = np.random.default_rng(seed + 1000)
    logit = np.log(scene.opacities.astype(np.float64)) - np.log1p(-scene.opacities.astype(np.float64))
    target = replace(scene,
                     means3d=(scene.means3d + rng.normal(0.0, 0.01, size=scene.means3d.shape)).astype(np.float32),
                     opacities=_sigmoid(logit + rng.normal(0.0, 0.2, size=n)).astype(np.float32))
    return scene, target, cams


def workload_fd(n: int = 64, seed: int = 5, size: int = 32):
    """Finite-difference sub-problem: the tiny generator with 64 splats, SH
    degree 3 (coefficients N(0, 0.3)) and a 32x32 camera."""
    return tiny_scene(n, seed=seed, sh_degree=3), tiny_camera(size, size)


def sample_pixels(width: int, height: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct pixels ([m, 2] int32 x, y) drawn uniformly."""
    rng = np.random.default_rng(seed)
    count = min(count, width * height)
    idx = rng.choice(width * height, size=count, replace=False)
    idx.sort()
    return np.stack([idx % width, idx // width], axis=1).astype(np.int32)


def binning_inputs(n: int, grid_w: int, grid_h: int, seed: int, culled: float = 0.1, ties: float = 0.2,
                   big: float = 0.003):
    """Seeded inputs of the binning stage alone, shaped like a projection's
    outputs: depth [n] float32 (positive; a fraction `ties` repeats another
    splat's depth, so equal keys occur), rect [n, 4] int32 tile rectangles
    (x0, y0, x1, y1) inside the grid, mostly one to a few tiles wide with a
    fraction `big` spanning up to the whole grid, and the empty rectangle
    (0, 0, -1, -1) for a fraction `culled`; tiles [n] uint32 = the rectangle's
    tile count."""
    rng = np.random.default_rng(seed)
    depth = rng.uniform(0.2, 120.0, n).astype(np.float32)
    if n > 1:
        tie = rng.random(n) < ties
        depth[tie] = depth[rng.integers(0, n, int(tie.sum()))]
    w = np.minimum(rng.geometric(0.45, n), grid_w)
    h = np.minimum(rng.geometric(0.45, n), grid_h)
    is_big = rng.random(n) < big
    w[is_big] = rng.integers(1, grid_w + 1, int(is_big.sum()))
    h[is_big] = rng.integers(1, grid_h + 1, int(is_big.sum()))
    x0 = (rng.random(n) * (grid_w - w + 1)).astype(np.int64)
    y0 = (rng.random(n) * (grid_h - h + 1)).astype(np.int64)
    rect = np.stack([x0, y0, x0 + w - 1, y0 + h - 1], axis=1)
    dead = rng.random(n) < culled
    rect[dead] = (0, 0, -1, -1)
    tiles = np.where(dead, 0, w * h).astype(np.uint32)
    return depth, rect.astype(np.int32), tiles


def thin_footprint_records(width: int, height: int, n: int = 12, seed: int = 7) -> dict:
    """Projected records (the float values, held as float64) of n footprints
    150-250 px long (standard deviation) and 0.4-1.2 px wide at angles spread
    over (0, pi), centred in the middle of the image, depths ascending in
    index order, each rectangle covering the whole tile grid. Near their axis
    the expanded terms of the quadratic form reach 1e5 while the form itself
    stays O(1). Keys: means2d, conic (a, b, c), opac, rgb, depth32, rect,
    flags."""
    rng = np.random.default_rng(seed)
    ang = np.linspace(0.1, math.pi - 0.1, n)
    s1, s2 = rng.uniform(150, 250, n), rng.uniform(0.4, 1.2, n)
    cs, sn = np.cos(ang), np.sin(ang)
    # inverse of R diag(s1^2, s2^2) R^T
    a = cs * cs / s1 ** 2 + sn * sn / s2 ** 2
    b = cs * sn * (1 / s1 ** 2 - 1 / s2 ** 2)
    c = sn * sn / s1 ** 2 + cs * cs / s2 ** 2
    gw, gh = (width + 15) // 16, (height + 15) // 16
    rec = dict(means2d=np.stack([rng.uniform(0.3, 0.7, n) * width, rng.uniform(0.3, 0.7, n) * height], 1),
               conic=np.stack([a, b, c], 1), opac=rng.uniform(0.5, 0.99, n), rgb=rng.uniform(0, 1, (n, 3)),
               depth32=np.sort(rng.uniform(1, 5, n)).astype(np.float32),
               rect=np.tile(np.array([0, 0, gw - 1, gh - 1], np.int32), (n, 1)), flags=np.zeros(n, np.uint8))
    for k in ("means2d", "conic", "opac", "rgb"):
        rec[k] = rec[k].astype(np.float32).astype(np.float64)
    return rec
