"""Seeded synthetic scenes, cameras and trajectories.

This module holds input recipes only: random draws of Gaussian parameters,
pinhole cameras and poses with the shapes and value distributions of the
workloads below.  It contains none of the rasterizer's arithmetic and is the
one place from which both the HIP path's tests/benchmarks and the CPU oracle
receive their inputs.

Workloads (the paper's datasets are not available; these stand in for its
1200-1600 px wide views with about one to two million primitives, section 5):

* ``tiny_scene``   -- one 128x128 pinhole view, fx=fy=128, principal point
  centred, identity pose, 2,000 Gaussians (means U([-1,1]^2 x [2,6]),
  log-scales N(-3, 0.5), random unit quaternions, opacity logits N(0,1),
  degree-0 colour U[0,1]) and a uniform random target image.
* ``ray_scene``    -- Gaussians placed along camera rays at depths from a
  smooth field (sum of four random sinusoids mapped to [1, 20]) plus N(0,0.02)
  jitter, SH degree 3 (DC ~ U[0,1], higher orders ~ N(0, 0.05)), a pixel
  footprint drawn from the distribution the paper's spawn rule produces
  (1/(2 sqrt(P)), P ~ U[0.05, 1], section 4.2) with N(0, 0.3) log jitter.
  Used at 1296x840 / 500k and at 1920x1080 / 2M (8 views x 250k).
* ``trajectory``   -- smooth random keyframe trajectory: per step a random
  axis with a 1-3 degree rotation and a 0.05-0.2 translation mostly along the
  viewing direction.

Arrays are float32 structure-of-arrays planes: means (3,N), log_scales (3,N),
quats (4,N) as (w,x,y,z), opacity_logits (N,), sh ((d+1)^2, 3, N).
Poses are world->camera (R row-major 3x3, t 3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Colour of a degree-0 SH coefficient c is 0.5 + c / (2 sqrt(pi)); this is
# the factor that maps a desired colour offset to its DC coefficient.
_DC_PER_COLOUR = 2.0 * math.sqrt(math.pi)


@dataclass
class View:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    R: np.ndarray = field(default_factory=lambda: np.eye(3))
    t: np.ndarray = field(default_factory=lambda: np.zeros(3))


@dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacity_logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.means.shape[1])

    def arrays(self):
        return dict(means=self.means, log_scales=self.log_scales, quats=self.quats,
                    opacity_logits=self.opacity_logits, sh=self.sh)


def _unit_quats(rng: np.random.Generator, n: int) -> np.ndarray:
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q.astype(np.float32)


def _rotation(axis: np.ndarray, angle: float) -> np.ndarray:
    a = axis / np.linalg.norm(axis)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * K @ K


def tiny_scene(seed: int = 0, n: int = 2000, size: int = 128):
    """The 128x128 / 2,000-Gaussian degree-0 scene and its L1 target."""
    rng = np.random.default_rng(seed)
    view = View(size, size, float(size), float(size), size / 2.0, size / 2.0)
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)]).astype(np.float32)
    log_scales = rng.normal(-3.0, 0.5, (3, n)).astype(np.float32)
    quats = _unit_quats(rng, n)
    opacity_logits = rng.normal(0.0, 1.0, n).astype(np.float32)
    rgb = rng.uniform(0, 1, (3, n))
    sh = ((rgb - 0.5) * _DC_PER_COLOUR).astype(np.float32)[None]
    target = rng.uniform(0, 1, (3, size, size)).astype(np.float32)
    return view, Scene(means, log_scales, quats, opacity_logits, sh, 0), target


def random_pose(rng: np.random.Generator, max_deg: float = 5.0, trans: float = 0.1):
    axis = rng.standard_normal(3)
    R = _rotation(axis, math.radians(rng.uniform(0.0, max_deg)))
    d = rng.standard_normal(3)
    t = trans * d / np.linalg.norm(d)
    return R, t


def _depth_field(rng, width, height, near=1.0, far=20.0):
    omega = rng.uniform(1, 6, (4, 2))
    phase = rng.uniform(0, 2 * math.pi, 4)

    def field_at(u, v):
        s = np.zeros_like(u, dtype=np.float64)
        for k in range(4):
            s += np.sin(2 * math.pi * (omega[k, 0] * u + omega[k, 1] * v) / width + phase[k])
        return near + (far - near) * (s + 4.0) / 8.0

    return field_at


def ray_points(rng, view: View, n: int, jitter: float = 0.02, depth_fn=None):
    """Points on random pixel rays of ``view`` at depths of a smooth field."""
    if depth_fn is None:
        depth_fn = _depth_field(rng, view.width, view.height)
    u = rng.uniform(0, view.width, n)
    v = rng.uniform(0, view.height, n)
    d = depth_fn(u, v)
    pc = np.stack([(u - view.cx) / view.fx * d, (v - view.cy) / view.fy * d, d])
    pw = view.R.T @ (pc - view.t[:, None])
    pw += rng.normal(0.0, jitter, pw.shape)
    return pw, d


def ray_scene(seed: int, view: View, n: int, sh_degree: int = 3, depth_fn=None, rng=None) -> Scene:
    rng = rng if rng is not None else np.random.default_rng(seed)
    means, d = ray_points(rng, view, n, depth_fn=depth_fn)
    f = math.sqrt(view.fx * view.fy)
    footprint_px = 1.0 / (2.0 * np.sqrt(rng.uniform(0.05, 1.0, n)))
    log_s = np.log(d * footprint_px / f)[None] + rng.normal(0.0, 0.3, (3, n))
    nb = (sh_degree + 1) ** 2
    sh = np.empty((nb, 3, n), np.float32)
    sh[0] = rng.uniform(0, 1, (3, n))
    if nb > 1:
        sh[1:] = rng.normal(0.0, 0.05, (nb - 1, 3, n))
    return Scene(means.astype(np.float32), log_s.astype(np.float32), _unit_quats(rng, n),
                 rng.normal(0.0, 1.0, n).astype(np.float32), sh, sh_degree)


def single_view(seed: int, width: int = 1296, height: int = 840, n: int = 500_000, sh_degree: int = 3):
    """One posed view (random 5 degree rotation, 0.1 translation), f = 0.7 W."""
    rng = np.random.default_rng(seed)
    f = 0.7 * width
    R, t = random_pose(rng)
    view = View(width, height, f, f, width / 2.0, height / 2.0, R, t)
    return view, ray_scene(seed, view, n, sh_degree, rng=rng)


def trajectory(seed: int, n_views: int, width: int, height: int):
    """Keyframes along a smooth random path (world->camera poses)."""
    rng = np.random.default_rng(seed)
    f = 0.7 * width
    views = []
    Rc = np.eye(3)  # camera->world rotation
    C = np.zeros(3)  # camera centre
    for _ in range(n_views):
        R = Rc.T
        views.append(View(width, height, f, f, width / 2.0, height / 2.0, R, -R @ C))
        dR = _rotation(rng.standard_normal(3), math.radians(rng.uniform(1.0, 3.0)))
        step = rng.uniform(0.05, 0.2)
        forward = Rc[:, 2]
        lateral = rng.standard_normal(3) * 0.2
        move = forward + lateral - forward * (forward @ lateral)
        C = C + step * move / np.linalg.norm(move)
        Rc = Rc @ dR
    return views


def window_scene(seed: int, views, per_view: int, sh_degree: int = 3) -> Scene:
    """Union of ray scenes, ``per_view`` Gaussians seeded from each keyframe."""
    rng = np.random.default_rng(seed + 7919)
    depth_fn = _depth_field(rng, views[0].width, views[0].height)
    parts = [ray_scene(0, v, per_view, sh_degree, depth_fn=depth_fn, rng=rng) for v in views]
    cat = lambda name, axis: np.concatenate([getattr(p, name) for p in parts], axis=axis)
    return Scene(cat("means", 1), cat("log_scales", 1), cat("quats", 1), cat("opacity_logits", 0),
                 cat("sh", 2), sh_degree)


def perturb_scene(seed: int, scene: Scene) -> Scene:
    """Optimisation start: ground truth plus noise on means/scales/colour/opacity."""
    rng = np.random.default_rng(seed + 104729)
    z = np.maximum(np.abs(scene.means[2]), 1.0)
    means = scene.means + rng.normal(0, 1, scene.means.shape) * (0.01 * z)
    log_s = scene.log_scales + rng.normal(0, 0.2, scene.log_scales.shape)
    sh = scene.sh.copy()
    sh[0] += rng.normal(0, 0.05, sh[0].shape)
    op = scene.opacity_logits + rng.normal(0, 0.5, scene.opacity_logits.shape)
    return Scene(means.astype(np.float32), log_s.astype(np.float32), scene.quats.copy(),
                 op.astype(np.float32), sh.astype(np.float32), scene.sh_degree)


def perturb_pose(rng, R: np.ndarray, t: np.ndarray, sigma: float = 0.01):
    """Left-multiply a pose by exp of a N(0, sigma^2) twist."""
    w = rng.normal(0, sigma, 3)
    dR = _rotation(w, np.linalg.norm(w)) if np.linalg.norm(w) > 0 else np.eye(3)
    return dR @ R, dR @ t + rng.normal(0, sigma, 3)


def small_scene(seed: int, n: int = 12, size: int = 32, sh_degree: int = 0, spread: float = 0.6):
    """A handful of well separated Gaussians for finite-difference checks."""
    rng = np.random.default_rng(seed)
    f = 1.1 * size
    view = View(size, size, f, f * 1.05, size / 2.0 + 0.3, size / 2.0 - 0.2)
    means = np.stack([rng.uniform(-spread, spread, n), rng.uniform(-spread, spread, n),
                      rng.uniform(2.0, 4.0, n)]).astype(np.float32)
    log_scales = rng.normal(-2.3, 0.3, (3, n)).astype(np.float32)
    quats = _unit_quats(rng, n)
    opacity_logits = rng.normal(0.0, 0.7, n).astype(np.float32)
    nb = (sh_degree + 1) ** 2
    sh = np.empty((nb, 3, n), np.float32)
    sh[0] = (rng.uniform(0.1, 0.9, (3, n)) - 0.5) * _DC_PER_COLOUR
    if nb > 1:
        sh[1:] = rng.normal(0.0, 0.3, (nb - 1, 3, n))
    return view, Scene(means, log_scales, quats, opacity_logits, sh, sh_degree)


def spawn_frame(seed: int, width: int = 1920, height: int = 1080, n_rects: int = 60, missing: float = 0.5):
    """A new frame for the spawn step (section 4.2): (image, rendered, depth).

    image [3][H][W] in [0,1]: a smooth background colour gradient, `n_rects`
    random axis-aligned rectangles of uniform random colour (sides
    U[2%, 30%] of the image, so edges at all scales), and N(0, 0.02) pixel
    noise clipped to [0, 1] (the sensor noise that gives every pixel a small
    P_L).  rendered: the same composition with a random `missing` fraction of
    the rectangles left out and no noise -- the model renders part of the
    frame's structure.  depth [H][W]: the smooth depth field of `ray_scene`
    in [1, 20], with each rectangle at its own constant depth U[1, 20]."""
    rng = np.random.default_rng(seed)
    H, W = height, width
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    base = np.stack([0.3 + 0.4 * x / max(W - 1, 1), 0.3 + 0.4 * y / max(H - 1, 1),
                     np.full((H, W), 0.5)])
    img, ren = base.copy(), base.copy()
    dz = _depth_field(rng, W, H)(x, y)
    keep = rng.random(n_rects) >= missing
    for i in range(n_rects):
        w = int(rng.uniform(0.02, 0.3) * W) + 1
        h = int(rng.uniform(0.02, 0.3) * H) + 1
        x0 = int(rng.integers(0, max(W - w, 1)))
        y0 = int(rng.integers(0, max(H - h, 1)))
        col = rng.random(3)
        img[:, y0:y0 + h, x0:x0 + w] = col[:, None, None]
        if keep[i]:
            ren[:, y0:y0 + h, x0:x0 + w] = col[:, None, None]
        dz[y0:y0 + h, x0:x0 + w] = rng.uniform(1.0, 20.0)
    img = np.clip(img + rng.normal(0, 0.02, img.shape), 0, 1)
    return img.astype(np.float32), ren.astype(np.float32), dz.astype(np.float32)


def mlp_init(seed: int, dims=(196, 64, 64, 7), last_scale: float = 0.1) -> np.ndarray:
    """Initial parameters of the spawn MLP, packed as (W1, b1, W2, b2, W3, b3)
    with W row-major [out][in]: W ~ N(0, 1/fan_in) (the last layer scaled by
    `last_scale`, so the untrained network starts near the rule), biases 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(len(dims) - 1):
        w = rng.standard_normal((dims[i + 1], dims[i])) / math.sqrt(dims[i])
        if i == len(dims) - 2:
            w *= last_scale
        parts += [w.ravel(), np.zeros(dims[i + 1])]
    return np.concatenate(parts).astype(np.float32)


def depth_frames(seed: int, width: int = 1920, height: int = 1080, channels: int = 32, n_nb: int = 2,
                 mono_err: float = 0.15):
    """Inputs of the guided-matching depth: frame i and n_nb neighbours
    looking at a tilted textured plane Z = z0 + a X + b Y (frame i's
    coordinates).  Features are random Fourier features of the plane point
    (X, Y) where each pixel's ray meets the plane, stored float16 [H][W][C];
    the monocular depth is the true depth times (1 + N(0, mono_err)).
    Returns (feat_i, [feat_j], rel_poses [n_nb][12], zmono, true depth, K)."""
    rng = np.random.default_rng(seed)
    f = 0.7 * width
    K = (f, f, (width - 1) / 2.0, (height - 1) / 2.0)
    z0, a, b = rng.uniform(3.0, 6.0), rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3)
    om = rng.normal(0.0, 2.0 * np.pi * f / (8.0 * z0), (channels, 2))  # texture periods of ~8 px at z0
    ph = rng.uniform(0.0, 2.0 * np.pi, channels)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64)
    rays = np.stack([(xx - K[2]) / K[0], (yy - K[3]) / K[1], np.ones_like(xx)], -1)
    nrm = np.array([-a, -b, 1.0])

    def view(R, t):
        # camera j: p_j = R p_i + t, so its centre is -R^T t and its rays R^T r in frame i
        o = -R.T @ t
        d = rays @ R  # (R^T r) for every pixel
        s = (z0 - nrm @ o) / (d @ nrm)
        P = o + s[..., None] * d
        phase = P[..., 0:1] * om[:, 0] + P[..., 1:2] * om[:, 1] + ph
        return (np.sqrt(2.0 / channels) * np.cos(phase)).astype(np.float16), P[..., 2]

    feat_i, z_true = view(np.eye(3), np.zeros(3))
    feats, poses = [], []
    for _ in range(n_nb):
        R = _rotation(rng.standard_normal(3), math.radians(rng.uniform(0.5, 3.0)))
        t = np.array([rng.uniform(-0.4, 0.4), rng.uniform(-0.1, 0.1), rng.uniform(-0.2, 0.2)])
        fj, _ = view(R, t)
        feats.append(fj)
        poses.append(np.concatenate([R.reshape(9), t]))
    zmono = (z_true * (1.0 + rng.normal(0.0, mono_err, z_true.shape))).astype(np.float32)
    return feat_i, feats, np.array(poses, np.float32), zmono, z_true, K
