"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This module draws random scenes, cameras, frame residuals and target images
with ``numpy.random.default_rng``. It holds none of the rasterizer's
arithmetic (no projection, compositing or rate computation): it only fixes
the shapes, distributions and structure of the workloads.

Parameter layout (planar, float32, ``[C][N]`` with ``C = 11 + 3 (d+1)^2``):

    0..2   mean (x, y, z)
    3..5   log-scale
    6..9   rotation quaternion (w, x, y, z), not necessarily unit length
    10     opacity logit
    11+3k+c  spherical-harmonic coefficient k, colour channel c

The Gaussian parameter set is the one of the 3D Gaussian representation in
Sec. 3.1 (centre, rotation, scales, opacity, SH coefficients).

Camera layout (float32 ``[16]`` per camera): a row-major world-to-camera
``[R | t]`` (12 values, OpenCV axes: x right, y down, z forward), then
``fx, fy, cx, cy``.

Residual layout (float32 ``[F][R][N]``): 0..2 translation delta, 3..6 rotation
delta quaternion (w, x, y, z), 7 opacity-logit delta, then optionally 8..10
log-scale delta and 11.. SH deltas; frame f composes the keyframe with the
deltas of frames 0..f (Sec. 3.2, pose update and Eq. 7).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# 1 / (2 sqrt(pi)): the constant degree-0 SH function. Used only so that a
# degree-0 colour drawn uniformly in [0, 1] can be stored as a coefficient.
_Y00 = 0.28209479177387814


def n_channels(sh_degree: int) -> int:
    return 11 + 3 * (sh_degree + 1) ** 2


def _unit_quats(rng, n):
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    return q


def _fill_common(rng, params, n, sh_degree, log_scale_mu=-3.0, log_scale_sd=0.5):
    params[3:6] = rng.normal(log_scale_mu, log_scale_sd, (3, n))
    params[6:10] = _unit_quats(rng, n)
    params[10] = rng.standard_normal(n)
    rgb = rng.uniform(0.0, 1.0, (3, n))
    params[11:14] = (rgb - 0.5) / _Y00
    k = (sh_degree + 1) ** 2
    if k > 1:
        params[14:11 + 3 * k] = rng.normal(0.0, 0.2, (3 * (k - 1), n))


def slab_scene(n: int, seed: int, sh_degree: int = 0) -> np.ndarray:
    """Means x, y ~ U[-1, 1], z ~ U[2, 6] in front of a camera at the origin."""
    rng = np.random.default_rng(seed)
    c = n_channels(sh_degree)
    p = np.zeros((c, n), np.float64)
    p[0] = rng.uniform(-1.0, 1.0, n)
    p[1] = rng.uniform(-1.0, 1.0, n)
    p[2] = rng.uniform(2.0, 6.0, n)
    _fill_common(rng, p, n, sh_degree)
    return np.ascontiguousarray(p.astype(np.float32))


def cube_scene(n: int, seed: int, sh_degree: int = 3) -> np.ndarray:
    """Means ~ U[-1, 1]^3 (a cloud seen by a camera ring), in generation order. The hierarchy's
    nested layers come from ordering the Gaussians by significance, which is the method's own
    step: the benchmark does it with the library, the tests with the oracle (see ``reorder``)."""
    rng = np.random.default_rng(seed)
    c = n_channels(sh_degree)
    p = np.zeros((c, n), np.float64)
    p[0:3] = rng.uniform(-1.0, 1.0, (3, n))
    _fill_common(rng, p, n, sh_degree)
    return np.ascontiguousarray(p.astype(np.float32))


def reorder(a: np.ndarray, order) -> np.ndarray:
    """The columns (last axis: Gaussians) of a parameter or residual array in the given order."""
    return np.ascontiguousarray(np.asarray(a)[..., np.asarray(order)])


def identity_camera(width: int, height: int, focal: float) -> np.ndarray:
    cam = np.zeros(16, np.float32)
    cam[0] = cam[5] = cam[10] = 1.0
    cam[12] = cam[13] = focal
    cam[14] = width / 2.0
    cam[15] = height / 2.0
    return cam


def look_at_camera(eye, target, down, width: int, height: int, focal: float) -> np.ndarray:
    """World-to-camera [R | t] for a pinhole at ``eye`` looking at ``target``."""
    eye = np.asarray(eye, np.float64)
    z = np.asarray(target, np.float64) - eye
    z /= np.linalg.norm(z)
    y = np.asarray(down, np.float64)
    y = y - z * np.dot(y, z)
    y /= np.linalg.norm(y)
    x = np.cross(y, z)
    r = np.stack([x, y, z])
    t = -r @ eye
    cam = np.zeros(16, np.float32)
    cam[0:12] = np.concatenate([r, t[:, None]], axis=1).reshape(-1)
    cam[12] = cam[13] = focal
    cam[14] = width / 2.0
    cam[15] = height / 2.0
    return cam


def ring_cameras(indices, n_ring: int = 24, radius: float = 4.0, width: int = 960,
                 height: int = 540, focal: float | None = None) -> np.ndarray:
    """Cameras at radius*(cos t, 0, sin t), t = 2 pi k / n_ring, looking at the origin, image-down = +y."""
    focal = float(width) if focal is None else focal
    cams = []
    for k in indices:
        th = 2.0 * math.pi * k / n_ring
        eye = (radius * math.cos(th), 0.0, radius * math.sin(th))
        cams.append(look_at_camera(eye, (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), width, height, focal))
    return np.ascontiguousarray(np.stack(cams))


def frame_residuals(n: int, n_frames: int, seed: int, channels: int = 8,
                    sd_mean: float = 0.01, sd_angle: float = 0.02, sd_logit: float = 0.05,
                    sd_log_scale: float = 0.0, sd_sh: float = 0.0) -> np.ndarray:
    """Per-frame deltas: translation N(0, sd_mean^2), rotation by an angle N(0, sd_angle) about a
    uniform axis (as a unit quaternion), opacity-logit N(0, sd_logit); optional log-scale / SH deltas."""
    rng = np.random.default_rng(seed)
    r = np.zeros((n_frames, channels, n), np.float64)
    for f in range(n_frames):
        r[f, 0:3] = rng.normal(0.0, sd_mean, (3, n))
        axis = rng.standard_normal((3, n))
        axis /= np.linalg.norm(axis, axis=0, keepdims=True)
        ang = rng.normal(0.0, sd_angle, n)
        r[f, 3] = np.cos(ang / 2)
        r[f, 4:7] = np.sin(ang / 2) * axis
        r[f, 7] = rng.normal(0.0, sd_logit, n)
        if channels > 8:
            r[f, 8:11] = rng.normal(0.0, sd_log_scale, (3, n)) if sd_log_scale > 0 else 0.0
        if channels > 11:
            r[f, 11:] = rng.normal(0.0, sd_sh, (channels - 11, n)) if sd_sh > 0 else 0.0
    return np.ascontiguousarray(r.astype(np.float32))


def target_images(n_images: int, width: int, height: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(0.0, 1.0, (n_images, 3, height, width)).astype(np.float32))


def motion_params(seed: int, table_floats: int, weight_shapes, table_scale: float = 1e-4):
    """Seeded parameters of a hash-grid + MLP motion network: a table of uniform values in
    [-table_scale, table_scale], He-normal weight matrices [out][in] and zero biases, flattened
    in the order of weight_shapes (2-tuples are matrices, 1-tuples biases)."""
    rng = np.random.default_rng(seed)
    table = rng.uniform(-table_scale, table_scale, table_floats).astype(np.float32)
    parts = []
    for s in weight_shapes:
        if len(s) == 2:
            parts.append(rng.normal(0.0, math.sqrt(2.0 / s[1]), s).ravel())
        else:
            parts.append(np.zeros(s).ravel())
    return table, np.concatenate(parts).astype(np.float32)


def loss_images(n_images: int, n_levels: int, width: int, height: int, seed: int):
    """Render-like colour layers and targets for the colour-loss path, float32 in [0, 1]:
    image [n_images][n_levels][3][height][width], target [n_images][3][height][width].

    The target is a few smooth colour blobs with fine texture over a flat background; every
    layer reproduces the background exactly (ties with the target, flat windows) and the blobs
    with detail and accuracy that grow with the layer index, like the nested layers of a
    hierarchy (no layer equals the target)."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float32) + 0.5
    img = np.empty((n_images, n_levels, 3, height, width), np.float32)
    tgt = np.empty((n_images, 3, height, width), np.float32)
    for b in range(n_images):
        field = np.zeros((3, height, width), np.float32)
        for _ in range(8):
            cx, cy = rng.uniform(0, width), rng.uniform(0, height)
            s = rng.uniform(2.0, 0.15 * max(width, height) + 2.0)
            amp = rng.uniform(0.1, 0.7, 3).astype(np.float32)
            field += amp[:, None, None] * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2.0 * s * s))
        fg = field.sum(axis=0) > 0.15
        bg = rng.uniform(0.0, 1.0, 3).astype(np.float32)[:, None, None]
        tex = rng.uniform(-0.15, 0.15, (3, height, width)).astype(np.float32)
        tgt[b] = np.where(fg, np.clip(bg * 0.3 + field + tex, 0.0, 1.0), bg)
        for l in range(n_levels):
            keep = (l + 1) / (n_levels + 1)
            err = rng.uniform(-0.05, 0.05, (3, height, width)).astype(np.float32) * (1.0 - keep)
            img[b, l] = np.where(fg, np.clip(bg * 0.3 + field + keep * tex + err, 0.0, 1.0), bg)
    return np.ascontiguousarray(img), np.ascontiguousarray(tgt)


@dataclasses.dataclass
class Workload:
    """One seeded workload: params, optional residuals, cameras [F*V][16], image size, levels."""
    name: str
    params: np.ndarray
    cams: np.ndarray
    width: int
    height: int
    sh_degree: int
    level_counts: list
    level_weights: list
    n_frames: int = 1
    residuals: np.ndarray | None = None
    target: np.ndarray | None = None

    @property
    def n(self) -> int:
        return self.params.shape[1]

    @property
    def n_views(self) -> int:
        return self.cams.shape[0] // self.n_frames


def paper_level_weights(n_levels: int):
    """0.5 / l for l < L and 1 for l = L (App. A, layer weights)."""
    return [0.5 / l for l in range(1, n_levels)] + [1.0]


def config_plain_forward(seed: int = 1, n: int = 4096, width: int = 128, height: int = 128) -> Workload:
    """4,096 Gaussians, 128x128, one camera at the origin looking +z, fx=fy=128, SH degree 0."""
    p = slab_scene(n, seed, 0)
    cams = identity_camera(width, height, 128.0 * width / 128.0)[None]
    return Workload("plain_forward_4096_128x128", p, cams, width, height, 0, [n], [1.0])


def config_forward_backward(seed: int = 2, n: int = 200_000, width: int = 1280, height: int = 720,
                            target_seed: int = 12) -> Workload:
    """200k Gaussians, SH degree 3, 1280x720, one camera (fx = fy = W), L1 to a uniform-noise target."""
    p = slab_scene(n, seed, 3)
    cams = identity_camera(width, height, float(width))[None]
    tgt = target_images(1, width, height, target_seed)
    return Workload(f"fwd_bwd_{n}_{width}x{height}", p, cams, width, height, 3, [n], [1.0], target=tgt)


LEVEL_FRACTIONS = (1 / 12, 2 / 12, 3 / 12, 6 / 12, 9 / 12, 1.0)  # 25k/50k/75k/150k/225k/300k of 300k


def nested_levels(n: int):
    return [int(round(n * f)) for f in LEVEL_FRACTIONS]


def config_batched(seed: int = 3, n: int = 300_000, n_views: int = 24, width: int = 960, height: int = 540,
                   target_seed: int = 13, view_indices=None) -> Workload:
    """300k Gaussians in a cube, a 24-camera ring of radius 4, 960x540, SH 3, six nested levels
    (prefixes of the Gaussians in the given order: sort them by significance first to make the
    levels the method's hierarchy)."""
    p = cube_scene(n, seed, 3)
    idx = list(range(n_views)) if view_indices is None else list(view_indices)
    cams = ring_cameras(idx, 24, 4.0, width, height)
    tgt = target_images(len(idx), width, height, target_seed)
    lv = nested_levels(n)
    return Workload(f"batched_{n}_{len(idx)}v_{width}x{height}_L6", p, cams, width, height, 3, lv,
                    paper_level_weights(6), target=tgt)


def config_group(seed: int = 4, n: int = 150_000, n_frames: int = 10, width: int = 960, height: int = 540,
                 target_seed: int = 14, view_indices=tuple(range(0, 24, 3))) -> Workload:
    """150k keyframe Gaussians, 10 residual frames, 8 ring views per frame."""
    p = cube_scene(n, seed, 3)
    res = frame_residuals(n, n_frames, seed + 100)
    cams1 = ring_cameras(view_indices, 24, 4.0, width, height)
    cams = np.ascontiguousarray(np.concatenate([cams1] * n_frames, axis=0))
    tgt = target_images(n_frames * len(view_indices), width, height, target_seed)
    return Workload(f"group_{n}_{n_frames}f_{len(view_indices)}v_{width}x{height}", p, cams, width, height, 3,
                    [n], [1.0], n_frames=n_frames, residuals=res, target=tgt)
