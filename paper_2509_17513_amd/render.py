"""Python binding of the render entry points: argument marshalling only.

Every step of the forward and backward runs in the HIP kernels of libgs4d.so;
torch provides the device memory and the stream.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import torch

from . import _lib
from ._lib import GsSettings, GsWorkspaceLayout, check, lib


@dataclasses.dataclass
class RenderSettings:
    width: int
    height: int
    sh_degree: int = 0
    level_counts: tuple = ()
    level_weights: tuple = ()
    res_channels: int = 0
    near_plane: float = 0.2
    dilation: float = 0.3
    alpha_min: float = 1.0 / 255.0
    alpha_max: float = 0.99
    t_stop: float = 1e-4
    bg: tuple = (0.0, 0.0, 0.0)
    # launch shapes (identical images for every value; see autotune): 0 = library default
    bin_chunk: int = 0
    row_seg: int = 0
    wave_layout: int = 0
    lds_batch: int = 0
    bwd_pixels: int = 0

    def c_struct(self, n: int) -> GsSettings:
        s = GsSettings()
        s.width, s.height, s.sh_degree = self.width, self.height, self.sh_degree
        lv = list(self.level_counts) if self.level_counts else [n]
        lw = list(self.level_weights) if self.level_weights else [1.0] * len(lv)
        if len(lv) > 8 or len(lw) != len(lv):
            raise ValueError("1..8 levels with one weight each")
        s.n_levels = len(lv)
        for i in range(len(lv)):
            s.level_counts[i] = int(lv[i])
            s.level_weights[i] = float(lw[i])
        s.res_channels = self.res_channels
        s.near_plane, s.dilation = self.near_plane, self.dilation
        s.alpha_min, s.alpha_max, s.t_stop = self.alpha_min, self.alpha_max, self.t_stop
        for i in range(3):
            s.bg[i] = self.bg[i]
        s.tile_w = s.tile_h = 0
        s.bin_chunk, s.row_seg, s.wave_layout = self.bin_chunk, self.row_seg, self.wave_layout
        s.lds_batch, s.bwd_pixels = self.lds_batch, self.bwd_pixels
        return s

    @property
    def n_levels(self):
        return max(1, len(self.level_counts))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(t, name, shape=None, dtype=torch.float32, device=None, min_numel=None):
    """Raises ValueError unless t is None or a contiguous CUDA tensor of this dtype, device and
    shape (the shape is checked first: the C ABI cannot see a tensor's extent)."""
    if t is None:
        return
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError(f"{name} needs at least {min_numel} elements")
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


class Workspace:
    """Device workspace of one render configuration. Grows when a forward reports that the
    (tile, Gaussian) pair list did not fit."""

    def __init__(self, settings: RenderSettings, n: int, n_frames: int, n_views: int, device,
                 pair_capacity: int | None = None):
        self.settings, self.n, self.F, self.V, self.device = settings, n, n_frames, n_views, device
        if pair_capacity is None:
            pair_capacity = max(1 << 16, 24 * n * n_frames * n_views)
        self.allocate(pair_capacity)

    def allocate(self, pair_capacity: int):
        pair_capacity = int(min(pair_capacity, (1 << 32) - 1))
        s = self.settings.c_struct(self.n)
        nbytes = ctypes.c_size_t()
        check(lib().gs_workspace_size(ctypes.byref(s), self.n, self.F, self.V, pair_capacity, ctypes.byref(nbytes)),
              "gs_workspace_size")
        self.pair_capacity = pair_capacity
        self.buf = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)

    @property
    def nbytes(self):
        return self.buf.numel()

    def layout(self) -> GsWorkspaceLayout:
        s = self.settings.c_struct(self.n)
        lo = GsWorkspaceLayout()
        check(lib().gs_workspace_describe(ctypes.byref(s), self.n, self.F, self.V, self.pair_capacity,
                                          ctypes.byref(lo)), "gs_workspace_describe")
        return lo

    def status(self):
        """(ok, needed_pairs); synchronises the current stream."""
        needed = ctypes.c_int64()
        rc = lib().gs_check_status(_ptr(self.buf), _stream(self.device), ctypes.byref(needed))
        if rc not in (_lib.GS_OK, _lib.GS_ERR_PAIR_OVERFLOW):
            check(rc, "gs_check_status")
        return rc == _lib.GS_OK, needed.value

    def stats(self) -> dict:
        """Work counters of the last raster passes on this workspace (synchronises the current
        stream); evals and contribs read 0 unless counting was on (``work_counters``)."""
        st = _lib.GsStats()
        check(lib().gs_workspace_stats(_ptr(self.buf), _stream(self.device), ctypes.byref(st)),
              "gs_workspace_stats")
        return {k: int(getattr(st, k)) for k in ("needed_pairs", "fwd_evals", "fwd_contribs", "bwd_evals",
                                                  "bwd_contribs")}


class deterministic:
    """Context in which workspaces are sized for, and backward passes run, the deterministic
    backward (gs_set_deterministic): the same gradient and loss bits on every run. Enter it before
    creating the workspace and running the forward."""

    def __enter__(self):
        self.prev = lib().gs_set_deterministic(1)
        return self

    def __exit__(self, *exc):
        lib().gs_set_deterministic(self.prev)
        return False


class work_counters:
    """Context in which raster passes run their work-counting variant (gs_set_work_counters)."""

    def __enter__(self):
        self.prev = lib().gs_set_work_counters(1)
        return self

    def __exit__(self, *exc):
        lib().gs_set_work_counters(self.prev)
        return False


def render_forward(settings: RenderSettings, params: torch.Tensor, cams: torch.Tensor, n_frames: int = 1,
                   residuals: torch.Tensor | None = None, ws: Workspace | None = None, image: torch.Tensor | None = None,
                   check_overflow: bool = True):
    """image [F][V][L][3][H][W]; returns (image, workspace)."""
    dev = params.device
    C = 11 + 3 * (settings.sh_degree + 1) ** 2
    n = params.shape[1]
    B = cams.shape[0]
    if params.dim() != 2 or params.shape[0] != C:
        raise ValueError(f"params must be [{C}][n]")
    if cams.dim() != 2 or cams.shape[1] != 16 or B % n_frames:
        raise ValueError("cams must be [n_frames * n_views][16]")
    V = B // n_frames
    _check_tensor(params, "params", device=dev)
    _check_tensor(cams, "cams", device=dev)
    if residuals is not None:
        _check_tensor(residuals, "residuals", (n_frames, settings.res_channels, n), device=dev)
    L = settings.n_levels
    shape = (n_frames, V, L, 3, settings.height, settings.width)
    if image is None:
        image = torch.empty(shape, dtype=torch.float32, device=dev)
    _check_tensor(image, "image", shape, device=dev)
    if ws is None:
        ws = Workspace(settings, n, n_frames, V, dev)
    s = settings.c_struct(n)
    for _ in range(3):
        check(lib().gs_render_forward(ctypes.byref(s), n, _ptr(params), n_frames, _ptr(residuals), V, _ptr(cams),
                                      _ptr(image), _ptr(ws.buf), ws.nbytes, _stream(dev)), "gs_render_forward")
        if not check_overflow:
            break
        ok, needed = ws.status()
        if ok:
            break
        ws.allocate(int(needed * 1.15) + 1024)
    else:
        raise RuntimeError("pair list kept overflowing")
    return image, ws


def render_backward(settings: RenderSettings, params: torch.Tensor, cams: torch.Tensor, ws: Workspace,
                    n_frames: int = 1, residuals: torch.Tensor | None = None, image: torch.Tensor | None = None,
                    d_image: torch.Tensor | None = None, target: torch.Tensor | None = None,
                    d_params: torch.Tensor | None = None, d_residuals: torch.Tensor | None = None,
                    loss: torch.Tensor | None = None):
    """Accumulates into d_params [C][n] (and d_residuals); returns (d_params, d_residuals)."""
    dev = params.device
    C = 11 + 3 * (settings.sh_degree + 1) ** 2
    if params.dim() != 2 or params.shape[0] != C:
        raise ValueError(f"params must be [{C}][n]")
    n = params.shape[1]
    if cams.dim() != 2 or cams.shape[1] != 16 or cams.shape[0] % n_frames:
        raise ValueError("cams must be [n_frames * n_views][16]")
    V = cams.shape[0] // n_frames
    H, W, L = settings.height, settings.width, settings.n_levels
    img_shape = (n_frames, V, L, 3, H, W)
    checks = ((d_image, "d_image", img_shape, None), (image, "image", img_shape, None),
              (target, "target", (n_frames * V, 3, H, W), None), (d_params, "d_params", (C, n), None),
              (residuals, "residuals", (n_frames, settings.res_channels, n), None),
              (d_residuals, "d_residuals", (n_frames, settings.res_channels, n), None), (loss, "loss", None, 1))
    for t, nm, shp, mn in checks:  # every extent first, then dtype, layout and device
        if t is not None and shp is not None and tuple(t.shape) != tuple(shp):
            raise ValueError(f"{nm} has shape {tuple(t.shape)}, expected {tuple(shp)}")
        if t is not None and mn is not None and t.numel() < mn:
            raise ValueError(f"{nm} needs at least {mn} elements")
    for t, nm, shp, mn in checks:
        _check_tensor(t, nm, shp, device=dev, min_numel=mn)
    if d_params is None:
        d_params = torch.zeros_like(params)
    if residuals is not None and d_residuals is None:
        d_residuals = torch.zeros_like(residuals)
    s = settings.c_struct(n)
    check(lib().gs_render_backward(ctypes.byref(s), n, _ptr(params), n_frames, _ptr(residuals), V, _ptr(cams),
                                   _ptr(image), _ptr(d_image), _ptr(target), _ptr(d_params), _ptr(d_residuals),
                                   _ptr(loss), _ptr(ws.buf), ws.nbytes, _stream(dev)), "gs_render_backward")
    return d_params, d_residuals


N_TUNE_TRIALS = 13
TUNED_FIELDS = ("bin_chunk", "row_seg", "wave_layout", "lds_batch", "bwd_pixels")


def autotune(settings: RenderSettings, params: torch.Tensor, cams: torch.Tensor, ws: Workspace, n_frames: int = 1,
             residuals: torch.Tensor | None = None, image: torch.Tensor | None = None):
    """Launch shapes for this workload (gs_autotune_render): returns (tuned settings, the thirteen
    trial times in ms per forward + backward, -1 for a trial whose image differed). The workspace
    must already hold the pairs (render once with check_overflow first)."""
    dev = params.device
    n = params.shape[1]
    B = cams.shape[0]
    if image is None:
        shape = (n_frames, B // n_frames, settings.n_levels, 3, settings.height, settings.width)
        image = torch.empty(shape, dtype=torch.float32, device=dev)
    dp = torch.zeros_like(params)
    dr = torch.zeros_like(residuals) if residuals is not None else None
    s = settings.c_struct(n)
    best = GsSettings()
    times = (ctypes.c_float * N_TUNE_TRIALS)()
    check(lib().gs_autotune_render(ctypes.byref(s), n, _ptr(params), n_frames, _ptr(residuals), B // n_frames,
                                   _ptr(cams), _ptr(image), _ptr(dp), _ptr(dr), _ptr(ws.buf), ws.nbytes, _stream(dev),
                                   ctypes.byref(best), times), "gs_autotune_render")
    tuned = dataclasses.replace(settings, **{f: getattr(best, f) for f in TUNED_FIELDS})
    return tuned, list(times)


def tune_cache_path() -> str:
    """The JSON tuning cache: $GS4D_TUNE_CACHE, else ~/.cache/gs4d/autotune.json."""
    return os.environ.get("GS4D_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "gs4d",
                                                             "autotune.json")


def tune_key(settings: RenderSettings, n: int, n_frames: int, n_views: int, device) -> str:
    """Cache key: the GPU architecture and every property of the workload the shapes depend on."""
    arch = torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]
    lv = ",".join(str(int(v)) for v in (settings.level_counts or (n,)))
    return (f"{arch}|n={n}|frames={n_frames}|views={n_views}|{settings.width}x{settings.height}|"
            f"sh={settings.sh_degree}|levels={lv}|res={settings.res_channels}")


def autotune_cached(settings: RenderSettings, params: torch.Tensor, cams: torch.Tensor, ws: Workspace,
                    n_frames: int = 1, residuals: torch.Tensor | None = None, image: torch.Tensor | None = None,
                    path: str | None = None):
    """autotune() through the JSON tuning cache: a workload already tuned on this architecture
    takes its stored shapes (no trials); otherwise the trials run and their winner is stored.
    Returns (tuned settings, trial times, True if the shapes came from the cache)."""
    import json
    path = path or tune_cache_path()
    key = tune_key(settings, params.shape[1], n_frames, cams.shape[0] // n_frames, params.device)
    try:
        with open(path) as fh:
            db = json.load(fh)
    except (OSError, ValueError):
        db = {}
    hit = db.get(key)
    if isinstance(hit, dict) and all(isinstance(hit.get(f), int) for f in TUNED_FIELDS):
        return dataclasses.replace(settings, **{f: hit[f] for f in TUNED_FIELDS}), hit.get("trial_ms"), True
    tuned, times = autotune(settings, params, cams, ws, n_frames, residuals, image)
    db[key] = {**{f: getattr(tuned, f) for f in TUNED_FIELDS}, "trial_ms": times}
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return tuned, times, False


class LossWorkspace:
    """Device workspace of gs_color_loss for one image shape (three floats per image element)."""

    def __init__(self, settings: RenderSettings, n_images: int, device):
        s = settings.c_struct(0 if not settings.level_counts else settings.level_counts[-1])
        nbytes = ctypes.c_size_t()
        check(lib().gs_color_loss_workspace_size(ctypes.byref(s), 1, n_images, ctypes.byref(nbytes)),
              "gs_color_loss_workspace_size")
        self.n_images = n_images
        self.buf = torch.empty(nbytes.value, dtype=torch.uint8, device=device)

    @property
    def nbytes(self):
        return self.buf.numel()


def color_loss(settings: RenderSettings, image: torch.Tensor, target: torch.Tensor, lambda_ssim: float,
               d_image: torch.Tensor | None = None, loss: torch.Tensor | None = None,
               ws: LossWorkspace | None = None, grad: bool = True):
    """Layer-weighted colour loss with its D-SSIM term (gs_color_loss).

    image [..., L, 3, H, W] (the render's output), target [..., 3, H, W] with the same leading
    images. Adds L to ``loss`` (one float) when given; returns dL/d image (for render_backward's
    d_image), or None when grad is False. Needs a GPU; every step runs in the library's kernels."""
    dev = image.device
    L, H, W = settings.n_levels, settings.height, settings.width
    if image.numel() % (L * 3 * H * W) or image.shape[-3:] != (3, H, W):
        raise ValueError(f"image of shape {tuple(image.shape)} is not [..., {L}, 3, {H}, {W}]")
    B = image.numel() // (L * 3 * H * W)
    _check_tensor(image, "image", device=dev)
    _check_tensor(target, "target", device=dev)
    if target.numel() != B * 3 * H * W:
        raise ValueError(f"target has {target.numel()} elements, expected {B} x 3 x {H} x {W}")
    if grad:
        if d_image is None:
            d_image = torch.empty_like(image)
        _check_tensor(d_image, "d_image", shape=image.shape, device=dev)
        if ws is None or ws.n_images != B:
            ws = LossWorkspace(settings, B, dev)
    else:
        d_image = None
        if loss is None:
            raise ValueError("nothing to compute: grad is False and loss is None")
    _check_tensor(loss, "loss", device=dev)
    s = settings.c_struct(0 if not settings.level_counts else settings.level_counts[-1])
    check(lib().gs_color_loss(ctypes.byref(s), 1, B, _ptr(image), _ptr(target), float(lambda_ssim), _ptr(d_image),
                              _ptr(loss), None if ws is None else _ptr(ws.buf), 0 if ws is None else ws.nbytes,
                              _stream(dev)), "gs_color_loss")
    return d_image


class RenderFunction(torch.autograd.Function):
    """Differentiable render: params (and residuals) -> image [F][V][L][3][H][W]."""

    @staticmethod
    def forward(ctx, params, residuals, cams, settings, n_frames):
        image, ws = render_forward(settings, params.detach(), cams, n_frames,
                                   None if residuals is None else residuals.detach())
        ctx.settings, ctx.n_frames, ctx.ws = settings, n_frames, ws
        ctx.save_for_backward(params, residuals, cams)
        return image

    @staticmethod
    def backward(ctx, d_image):
        params, residuals, cams = ctx.saved_tensors
        dp, dr = render_backward(ctx.settings, params.detach(), cams, ctx.ws, ctx.n_frames,
                                 None if residuals is None else residuals.detach(),
                                 d_image=d_image.contiguous())
        return dp, dr, None, None, None


def render(params, cams, settings: RenderSettings, n_frames: int = 1, residuals=None):
    return RenderFunction.apply(params, residuals, cams, settings, n_frames)
