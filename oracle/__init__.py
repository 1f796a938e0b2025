"""FP64 CPU oracle of the differentiable Gaussian rasterizer and of the rate terms.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg. The product library never imports it and it
shares no code with the GPU path (no kernels, headers, helpers or tables).

The rasterizer part is C++ (``gs_oracle.cpp``, FP64, OpenMP), loaded through
ctypes; see that file's header for the conventions it follows. The rate part
(``oracle.rate``) is NumPy in float64.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "gs_oracle.cpp")
_lib = None

N_VAR_MAX = 16


def build(force: bool = True) -> str:
    """Compile liboracle.so with g++ (FP64, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Settings(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("sh_degree", ctypes.c_int32),
        ("n_levels", ctypes.c_int32), ("level_counts", ctypes.c_int32 * 8), ("res_channels", ctypes.c_int32),
        ("pad_", ctypes.c_int32), ("near_plane", ctypes.c_double), ("dilation", ctypes.c_double),
        ("alpha_min", ctypes.c_double), ("alpha_max", ctypes.c_double), ("t_stop", ctypes.c_double),
        ("bg", ctypes.c_double * 3), ("band_safety", ctypes.c_double),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        L.oc_project.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, P]
        L.oc_render.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int,
                                ctypes.c_int64, P, P, P, P, P, P, P]
        L.oc_backward.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, P, P, P]
        L.oc_backward_abs.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P, P, P]
        L.oc_backward_abs.restype = ctypes.c_int
        L.oc_fd.argtypes = [P, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_int64, P, P, ctypes.c_double, P, P, P]
        L.oc_fd.restype = ctypes.c_int
        L.oc_set_threads.argtypes = [ctypes.c_int]
        L.oc_set_threads.restype = ctypes.c_int
        L.oc_sh_basis.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double, P]
        L.oc_quat_rot.argtypes = [P, P]
        L.oc_quat_mul.argtypes = [P, P, P]
        for f in (L.oc_project, L.oc_render, L.oc_backward):
            f.restype = ctypes.c_int
        _lib = L
    return _lib


@dataclasses.dataclass
class Settings:
    """Render settings. Every float is rounded to float32 before use, so that the oracle
    evaluates the same mathematical function as a float32-parameterised caller."""
    width: int
    height: int
    sh_degree: int = 0
    level_counts: tuple = ()
    near_plane: float = 0.2
    dilation: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_stop: float = 1e-4
    bg: tuple = (0.0, 0.0, 0.0)
    res_channels: int = 0
    # multiplier of the first-order float32 error bounds inside which a decision is
    # explored both ways (ambiguous pixels); 0 turns the exploration off
    band_safety: float = 2.0

    def c_struct(self, n: int) -> _Settings:
        s = _Settings()
        s.width, s.height, s.sh_degree = self.width, self.height, self.sh_degree
        lv = list(self.level_counts) if self.level_counts else [n]
        s.n_levels = len(lv)
        for i, v in enumerate(lv):
            s.level_counts[i] = int(v)
        s.res_channels = self.res_channels
        f32 = lambda x: float(np.float32(x))  # noqa: E731
        s.near_plane, s.dilation = f32(self.near_plane), f32(self.dilation)
        s.alpha_min, s.alpha_max, s.t_stop = f32(self.alpha_min), f32(self.alpha_max), f32(self.t_stop)
        for i in range(3):
            s.bg[i] = f32(self.bg[i])
        s.band_safety = self.band_safety
        return s


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _frames_views(cams, n_frames):
    B = cams.shape[0]
    assert B % n_frames == 0
    return n_frames, B // n_frames


def project(st: Settings, params, cams, n_frames=1, residuals=None):
    """Per (frame-view, Gaussian) projection, shape [B][N][16]:
    valid, depth key, mx, my, cov xx, xy, yy, conic A, B, C, opacity, r, g, b, radius, flags."""
    params, cams, residuals = _f32(params), _f32(cams), _f32(residuals)
    n = params.shape[1]
    F, V = _frames_views(cams, n_frames)
    out = np.zeros((F * V, n, 16), np.float64)
    s = st.c_struct(n)
    rc = lib().oc_project(ctypes.byref(s), n, _ptr(params), F, _ptr(residuals), V, _ptr(cams), _ptr(out))
    assert rc == 0
    return out


def render(st: Settings, params, cams, n_frames=1, residuals=None, mode="bucket", sample=None,
           variants=False, signature=False):
    """Render every frame-view and level. Returns a dict with
    image [B][L][3][H][W] (or [B][L][3][S] for a pixel sample), T [B][L][...], ncontrib,
    and optionally nvar / var (accepted alternative colours of ambiguous pixels) and sig."""
    params, cams, residuals = _f32(params), _f32(cams), _f32(residuals)
    n = params.shape[1]
    F, V = _frames_views(cams, n_frames)
    B = F * V
    s = st.c_struct(n)
    L = s.n_levels
    if sample is not None:
        sample = np.ascontiguousarray(sample, dtype=np.int64)
        npix = sample.shape[0]
        shp = (npix,)
    else:
        npix = st.width * st.height
        shp = (st.height, st.width)
    image = np.zeros((B, L, 3, npix), np.float64)
    T = np.zeros((B, L, npix), np.float64)
    nc = np.zeros((B, L, npix), np.int32)
    sig = np.zeros((B, L, npix), np.uint64) if signature else None
    nvar = np.zeros((B, L, npix), np.int32) if variants else None
    var = np.zeros((B, L, npix, N_VAR_MAX, 3), np.float64) if variants else None
    m = {"bucket": 0, "brute": 1}[mode]
    rc = lib().oc_render(ctypes.byref(s), n, _ptr(params), F, _ptr(residuals), V, _ptr(cams), m,
                         npix if sample is not None else 0, _ptr(sample), _ptr(image), _ptr(T), _ptr(nc),
                         _ptr(sig), _ptr(nvar), _ptr(var))
    assert rc == 0
    out = {"image": image.reshape((B, L, 3) + shp), "T": T.reshape((B, L) + shp),
           "ncontrib": nc.reshape((B, L) + shp)}
    if signature:
        out["sig"] = sig.reshape((B, L) + shp)
    if variants:
        out["nvar"] = nvar.reshape((B, L) + shp)
        out["var"] = var.reshape((B, L) + shp + (N_VAR_MAX, 3))
    return out


def backward(st: Settings, params, cams, d_image, n_frames=1, residuals=None, mode="bucket"):
    """Analytic FP64 gradient of sum(d_image * image). Returns (d_params [C][N], d_res or None,
    grad2d [B][N][9])."""
    params, cams, residuals = _f32(params), _f32(cams), _f32(residuals)
    n = params.shape[1]
    F, V = _frames_views(cams, n_frames)
    B = F * V
    s = st.c_struct(n)
    d_image = np.ascontiguousarray(d_image, dtype=np.float64)
    assert d_image.size == B * s.n_levels * 3 * st.width * st.height
    C = params.shape[0]
    dp = np.zeros((C, n), np.float64)
    dr = np.zeros_like(residuals, dtype=np.float64) if residuals is not None and st.res_channels > 0 else None
    g2 = np.zeros((B, n, 9), np.float64)
    m = {"bucket": 0, "brute": 1}[mode]
    rc = lib().oc_backward(ctypes.byref(s), n, _ptr(params), F, _ptr(residuals), V, _ptr(cams), m,
                           _ptr(d_image), _ptr(dp), _ptr(dr), _ptr(g2))
    assert rc == 0
    return dp, dr, g2


def backward_abs(st: Settings, params, cams, d_image, mode="bucket"):
    """(d_params, d_params_abs) for one frame without residuals: the analytic gradient of
    sum(d_image * image) and the same sums taken of the absolute values of their terms (per-pixel
    terms, then the projection Jacobian), the scale of the float32 rounding error of a gradient
    whose terms cancel."""
    params, cams = _f32(params), _f32(cams)
    n = params.shape[1]
    V = cams.shape[0]
    s = st.c_struct(n)
    d_image = np.ascontiguousarray(d_image, dtype=np.float64)
    assert d_image.size == V * s.n_levels * 3 * st.width * st.height
    C = params.shape[0]
    dp = np.zeros((C, n), np.float64)
    da = np.zeros((C, n), np.float64)
    m = {"bucket": 0, "brute": 1}[mode]
    rc = lib().oc_backward_abs(ctypes.byref(s), n, _ptr(params), V, _ptr(cams), m, _ptr(d_image), _ptr(dp), _ptr(da))
    assert rc == 0
    return dp, da


def finite_differences(st: Settings, params, cams, d_image, gauss, chan, h=1e-5):
    """FP64 central differences of sum(d_image * image) with respect to params[chan[j], gauss[j]],
    re-compositing only the perturbed Gaussian's footprint (one frame, every view and level).
    Returns (fd [m], status [m], skipped [m]); status bits: 1 one-sided difference used at some
    pixel-level, 2 step h/10 used, 4 some pixel-level skipped (kinked on both sides), 8 invalid."""
    params, cams = _f32(params), _f32(cams)
    n = params.shape[1]
    V = cams.shape[0]
    s = st.c_struct(n)
    d_image = np.ascontiguousarray(d_image, dtype=np.float64)
    assert d_image.size == V * s.n_levels * 3 * st.width * st.height
    gauss = np.ascontiguousarray(gauss, np.int32)
    chan = np.ascontiguousarray(chan, np.int32)
    m = gauss.shape[0]
    fd = np.zeros(m, np.float64)
    status = np.zeros(m, np.int32)
    skipped = np.zeros(m, np.int64)
    rc = lib().oc_fd(ctypes.byref(s), n, _ptr(params), V, _ptr(cams), _ptr(d_image), m, _ptr(gauss), _ptr(chan),
                     float(h), _ptr(fd), _ptr(status), _ptr(skipped))
    assert rc == 0
    return fd, status, skipped


def set_threads(n: int) -> int:
    """OpenMP threads of the C++ oracle's following calls; returns the previous count."""
    return int(lib().oc_set_threads(int(n)))


def sh_basis(deg: int, d) -> np.ndarray:
    out = np.zeros(16, np.float64)
    lib().oc_sh_basis(deg, float(d[0]), float(d[1]), float(d[2]), _ptr(out))
    return out[: (deg + 1) ** 2]


def quat_rot(q) -> np.ndarray:
    q = np.ascontiguousarray(q, np.float64)
    out = np.zeros(9, np.float64)
    lib().oc_quat_rot(_ptr(q), _ptr(out))
    return out.reshape(3, 3)


def quat_mul(a, b) -> np.ndarray:
    a = np.ascontiguousarray(a, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    out = np.zeros(4, np.float64)
    lib().oc_quat_mul(_ptr(a), _ptr(b), _ptr(out))
    return out


def l1_grad(image, target, level_weights):
    """dL/dC for L = sum_{b,l} lambda^l * mean_{pixel, channel} |C^l - target_b| (Sec. 3.3 colour
    term with the layer weights of the keyframe loss; D-SSIM weight 0). image [B][L][3][H][W]."""
    B, L, _, H, W = image.shape
    w = np.asarray(level_weights, np.float64).reshape(1, L, 1, 1, 1)
    return w * np.sign(image - target[:, None].astype(np.float64)) / (3.0 * H * W)


def l1_loss(image, target, level_weights):
    B, L, _, H, W = image.shape
    w = np.asarray(level_weights, np.float64)
    per = np.abs(image - target[:, None].astype(np.float64)).mean(axis=(2, 3, 4))  # [B][L]
    return float((per * w[None]).sum())
