"""Joint training of Gaussians and the learned rate model, on the library's kernels.

One step (every compute step is a C-ABI call into libgs4d.so; torch only holds memory):
  forward render of all views and layers -> fused layer-weighted L1 backward into d_params
  -> context features -> learned rate in training mode (uniform-noise quantisation; the rate
  gradient lands directly in the attribute rows of d_params, the maximum-likelihood fit of the
  entropy model in d_w, d_b) -> Adam on the parameter groups and on the MLP (FP32 masters with
  BF16 copies for the MFMA).

This is the keyframe objective of Sec. 3.3: sum_l lambda^l (L1^l + lambda_rate R^l) with the
D-SSIM weight 0 and the learned Laplace model as the differentiable rate.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import _lib
from ._lib import check, lib
from .render import LossWorkspace, RenderSettings, Workspace, color_loss, render_backward, render_forward

W_PER_ATTR = 16 * 64 + 64 * 64 + 2 * 64
B_PER_ATTR = 64 + 64 + 2
CTX_DIM = 16


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _off(t, elems):
    """Pointer elems float32 elements into t."""
    return ctypes.c_void_p(t.data_ptr() + 4 * elems)


def zero(t):
    check(lib().gs_zero(_p(t), t.numel() * t.element_size(), _s(t.device)), "gs_zero")


class Adam:
    """Adam state of one float32 device tensor; slices of it can be stepped with their own rate."""

    def __init__(self, param: torch.Tensor, betas=(0.9, 0.999), eps=1e-15):
        self.p = param
        self.m = torch.zeros_like(param)
        self.v = torch.zeros_like(param)
        self.b1, self.b2 = betas
        self.eps = eps

    def step(self, grad: torch.Tensor, lr: float, t: int, start: int = 0, count: int | None = None,
             bf16_copy: torch.Tensor | None = None, t_dev: torch.Tensor | None = None):
        """One Adam update with step number t, or with the step number held in the device int32
        t_dev (read when the kernel runs: a captured step replays with the right corrections)."""
        count = self.p.numel() - start if count is None else count
        cp = None if bf16_copy is None else ctypes.c_void_p(bf16_copy.data_ptr() + 2 * start)
        args = (count, _off(self.p, start), _off(grad, start), _off(self.m, start), _off(self.v, start), cp,
                ctypes.c_float(lr), ctypes.c_float(self.b1), ctypes.c_float(self.b2), ctypes.c_float(self.eps))
        if t_dev is None:
            check(lib().gs_adam_step(*args, t, _s(self.p.device)), "gs_adam_step")
        else:
            check(lib().gs_adam_step_dev(*args, _p(t_dev), _s(self.p.device)), "gs_adam_step_dev")


def _bf16_bits(x: np.ndarray) -> np.ndarray:
    """float64 -> BF16 bit patterns, round to nearest even (host-side initialisation only)."""
    u = x.astype(np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


class RateModel:
    """Per-attribute Laplace MLP (16 -> 64 -> 64 -> 2): FP32 masters, BF16 copies, Adam state."""

    def __init__(self, n_attr: int, device, seed: int = 0, attrs: torch.Tensor | None = None,
                 step: float = 1.0 / 64):
        """Seeded random weights (scaled by 1/sqrt(fan-in), the output layer 10x smaller) and zero
        biases; with attrs [n_attr][n] (device) the output bias starts at the context-free Laplace
        fit of each attribute (gs_rate_init_output_bias)."""
        rng = np.random.default_rng(seed)
        w = np.zeros((n_attr, W_PER_ATTR))
        w[:, :1024] = rng.standard_normal((n_attr, 1024)) * 0.25
        w[:, 1024:5120] = rng.standard_normal((n_attr, 4096)) * 0.125
        w[:, 5120:] = rng.standard_normal((n_attr, 128)) * 0.0125
        b = np.zeros((n_attr, B_PER_ATTR), np.float32)
        self.n_attr, self.step_size = n_attr, step
        self.w = torch.from_numpy(w.astype(np.float32)).to(device)
        self.w16 = torch.from_numpy(_bf16_bits(w).view(np.int16)).to(device)
        self.b = torch.from_numpy(b).to(device)
        self.dw = torch.zeros_like(self.w)
        self.db = torch.zeros_like(self.b)
        self.opt_w = Adam(self.w)
        self.opt_b = Adam(self.b)
        self.bits = torch.zeros(n_attr, dtype=torch.float64, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.t = 0
        self.blocks = 0  # launch blocks per attribute; 0 = library default (see autotune)
        if attrs is not None:
            self.init_output_bias(attrs)

    def init_output_bias(self, attrs: torch.Tensor):
        if tuple(attrs.shape[:1]) != (self.n_attr,) or not attrs.is_contiguous() or attrs.dtype != torch.float32:
            raise ValueError("attrs must be a contiguous float32 [n_attr][n] tensor")
        acc = torch.empty(2 * self.n_attr, dtype=torch.float64, device=self.b.device)
        check(lib().gs_rate_init_output_bias(attrs.shape[1], self.n_attr, _p(attrs), ctypes.c_float(self.step_size),
                                             _p(self.b), _p(acc), _s(self.b.device)), "gs_rate_init_output_bias")

    def desc(self, n, mode, level_counts, level_weights, lambda_rate, seed=0, offset=0, fit_scale=None,
             offset_dev=None):
        d = _lib.GsRateDesc()
        d.offset_dev = None if offset_dev is None else offset_dev.data_ptr()
        d.n, d.n_attr, d.step, d.mode, d.seed, d.offset = n, self.n_attr, self.step_size, mode, seed, offset
        d.n_levels = len(level_counts)
        for i, v in enumerate(level_counts):
            d.level_counts[i] = int(v)
            d.level_weights[i] = float(level_weights[i])
        d.lambda_rate = lambda_rate
        d.fit_scale = (1.0 / max(n, 1)) if fit_scale is None else fit_scale
        d.blocks_per_attr = self.blocks
        return d

    def run(self, attrs_ptr, n, ctx, mode, level_counts, level_weights, lambda_rate=0.0, seed=0, offset=0,
            d_attrs_ptr=None, grads=True, sym_bits=None, offset_dev=None):
        """Accumulates bits / loss (and gradients) of one pass; zero them first with reset().
        offset_dev: a device uint64 holding the noise counter offset (instead of offset)."""
        d = self.desc(n, mode, level_counts, level_weights, lambda_rate, seed, offset, offset_dev=offset_dev)
        check(lib().gs_rate_model(ctypes.byref(d), attrs_ptr, _p(ctx), _p(self.w16), _p(self.b), _p(self.bits),
                                  _p(self.loss), _p(sym_bits), d_attrs_ptr, _p(self.dw) if grads else None,
                                  _p(self.db) if grads else None, _s(self.w.device)), "gs_rate_model")

    def autotune(self, attrs_ptr, n, ctx, mode, level_counts, level_weights, lambda_rate=0.0, d_attrs_ptr=None,
                 grads=True):
        """Picks the launch shape (blocks per attribute) for this workload with gs_rate_autotune; the
        gradient buffers used for the timed calls are zeroed afterwards. Returns (blocks, times_ms)."""
        d = self.desc(n, mode, level_counts, level_weights, lambda_rate)
        scratch = torch.zeros((5, self.n_attr), dtype=torch.float64, device=self.w.device)
        best = ctypes.c_int32()
        times = (ctypes.c_float * 5)()
        check(lib().gs_rate_autotune(ctypes.byref(d), attrs_ptr, _p(ctx), _p(self.w16), _p(self.b), _p(scratch),
                                     d_attrs_ptr, _p(self.dw) if grads else None, _p(self.db) if grads else None,
                                     _s(self.w.device), ctypes.byref(best), times), "gs_rate_autotune")
        zero(self.dw)
        zero(self.db)
        self.blocks = int(best.value)
        return self.blocks, list(times)

    def reset(self):
        zero(self.bits)
        zero(self.loss)

    def adam(self, lr: float, t_dev: torch.Tensor | None = None):
        self.t += 1
        self.opt_w.step(self.dw, lr, self.t, bf16_copy=self.w16, t_dev=t_dev)
        self.opt_b.step(self.db, lr, self.t, t_dev=t_dev)


def context(params: torch.Tensor, extent: float, level_counts, out: torch.Tensor | None = None):
    n = params.shape[1]
    if out is None:
        out = torch.zeros((n, CTX_DIM), dtype=torch.int16, device=params.device)
    lv = (ctypes.c_int32 * len(level_counts))(*[int(v) for v in level_counts])
    check(lib().gs_rate_context(n, _p(params), ctypes.c_float(extent), len(level_counts), lv, _p(out),
                                _s(params.device)), "gs_rate_context")
    return out


def histogram_bits(attrs: torch.Tensor, step: float = 1.0 / 64, ws: torch.Tensor | None = None):
    """Per-attribute empirical-histogram rate (float64 bits) of attrs [A][n] (synchronises)."""
    A, n = attrs.shape
    sz = ctypes.c_size_t()
    check(lib().gs_rate_histogram_workspace_size(A, ctypes.byref(sz)), "gs_rate_histogram_workspace_size")
    if ws is None or ws.numel() < sz.value:
        ws = torch.zeros(sz.value, dtype=torch.uint8, device=attrs.device)
    bits = torch.zeros(A, dtype=torch.float64, device=attrs.device)
    check(lib().gs_rate_histogram(n, A, _p(attrs), ctypes.c_float(step), _p(bits), _p(ws), ws.numel(),
                                  _s(attrs.device)), "gs_rate_histogram")
    return bits


@dataclasses.dataclass
class LearningRates:
    """Per-group Adam rates of the Gaussian parameters (3DGS-style) and of the rate MLP."""
    mean: float = 1.6e-4
    log_scale: float = 5e-3
    quat: float = 1e-3
    logit: float = 5e-2
    sh_dc: float = 2.5e-3
    sh_rest: float = 2.5e-3 / 20
    mlp: float = 2e-3


class JointTrainer:
    """Keyframe training on all views and layers at once: the layer-weighted colour loss (L1, plus
    D-SSIM when lambda_ssim > 0) and a rate term: the learned rate (`rate`), or the paper's own KDE
    rate of the attributes (`kde_rate=True`, Sec. 3.3: the keyframe objective
    sum_l lambda^l (L_color^l + lambda_rate L_rate^l) with the Silverman-bandwidth KDE)."""

    def __init__(self, params: torch.Tensor, cams: torch.Tensor, targets: torch.Tensor, settings: RenderSettings,
                 rate: RateModel | None, lambda_rate: float = 0.0, extent: float = 1.0,
                 lrs: LearningRates | None = None, seed: int = 0, lambda_ssim: float = 0.0, kde_rate: bool = False,
                 check_every: int = 1):
        self.p, self.cams, self.tgt, self.st = params, cams, targets, settings
        # the pair-list status is read after the forward every check_every steps: an overflow grows
        # the workspace and redoes the forward before any gradient is taken (1 = every step; with
        # more, a step between two checks may compute its colour gradient from a stale image)
        self.check_every = max(1, int(check_every))
        self.n = params.shape[1]
        self.rate, self.lam, self.extent = rate, lambda_rate, extent
        self.lrs = lrs or LearningRates()
        self.dp = torch.zeros_like(params)
        self.opt = Adam(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        self.ctx = torch.zeros((self.n, CTX_DIM), dtype=torch.int16, device=params.device)
        self.t = 0
        self.seed = seed
        self.img, self.ws = render_forward(settings, params, cams)  # sizes the workspace
        self.levels = list(settings.level_counts) if settings.level_counts else [self.n]
        self.level_w = list(settings.level_weights) if settings.level_weights else [1.0] * len(self.levels)
        self.lambda_ssim = lambda_ssim
        self.kde = None
        if kde_rate:
            from .entropy import KDE, EntropyModel
            A = params.shape[0] - 3
            self.kde = EntropyModel(A, self.n, KDE, params.device, 1.0 / 64, self.levels, self.level_w, lambda_rate)
            self.kde_loss = torch.zeros(1, dtype=torch.float64, device=params.device)
        if lambda_ssim > 0:
            self.d_img = torch.empty_like(self.img)
            self.loss_ws = LossWorkspace(settings, cams.shape[0], params.device)

    def step(self, check_overflow: bool | None = None):
        if check_overflow is None:
            check_overflow = self.t % self.check_every == 0
        self._forward(check_overflow)
        self._rest()

    def _forward(self, check_overflow=False):
        zero(self.loss)
        render_forward(self.st, self.p, self.cams, ws=self.ws, image=self.img, check_overflow=check_overflow)

    def _rest(self, counters=None):
        """Everything after the forward render. counters = (t_dev, off_dev): the step number and
        the rate's noise offset are taken from (and advanced in) device memory, for capture."""
        n = self.n
        if self.lambda_ssim > 0:
            color_loss(self.st, self.img, self.tgt, self.lambda_ssim, d_image=self.d_img, loss=self.loss,
                       ws=self.loss_ws)
            render_backward(self.st, self.p, self.cams, self.ws, d_image=self.d_img, d_params=self.dp)
        else:
            render_backward(self.st, self.p, self.cams, self.ws, image=self.img, target=self.tgt, d_params=self.dp,
                            loss=self.loss)
        t_dev, off_dev = counters if counters is not None else (None, None)
        if self.rate is not None:
            self.rate.reset()
            context(self.p, self.extent, self.levels, self.ctx)
            A = self.rate.n_attr
            self.rate.run(_off(self.p, 3 * n), n, self.ctx, 1, self.levels, self.level_w, self.lam,
                          seed=self.seed, offset=self.t * A * n,
                          d_attrs_ptr=_off(self.dp, 3 * n) if self.lam > 0 else None, offset_dev=off_dev)
        if counters is not None:
            A = self.rate.n_attr if self.rate is not None else 0
            check(lib().gs_advance_counters(_p(t_dev), _p(off_dev), A * n, _s(self.p.device)), "gs_advance_counters")
        if self.rate is not None:
            self.rate.adam(self.lrs.mlp, t_dev=t_dev)
        if self.kde is not None:
            # the rate of the attribute rows (everything but the means), noisy symbols, its
            # gradient added into the same rows of d_params
            zero(self.kde_loss)
            self.kde.run(self.p[3:], 1, seed=self.seed, offset=self.t * self.kde.desc.n_attr * n,
                         loss=self.kde_loss, d_attrs=self.dp[3:])
        self.t += 1
        K = self.p.shape[0] - 11
        lr = self.lrs
        for lo, hi, r in ((0, 3, lr.mean), (3, 6, lr.log_scale), (6, 10, lr.quat), (10, 11, lr.logit),
                          (11, 14, lr.sh_dc), (14, 11 + K, lr.sh_rest)):
            if hi > lo:
                self.opt.step(self.dp, r, self.t, start=lo * n, count=(hi - lo) * n, t_dev=t_dev)

    def capture(self):
        """Captures one training step in two hipGraphs (torch.cuda.CUDAGraph): the forward render,
        and everything after it (colour loss backward, context, learned rate with its gradient, the
        Adams), with the step number and the rate's noise offset in device counters that the graph
        advances, so that replays (step_graph) train exactly like eager steps. The KDE rate is not
        captured (its noise offset is a host argument)."""
        if self.kde is not None:
            raise ValueError("the KDE rate path is not captured")
        dev = self.p.device
        A = self.rate.n_attr if self.rate is not None else 0
        self.t_dev = torch.tensor([self.t], dtype=torch.int32, device=dev)
        self.off_dev = torch.tensor([self.t * A * self.n], dtype=torch.int64, device=dev)
        if self.rate is not None:
            self.rate.t = self.t
        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        self.g_fwd, self.g_rest = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.g_fwd, stream=side):
            self._forward(False)
        t0 = self.t
        with torch.cuda.graph(self.g_rest, stream=side):
            self._rest((self.t_dev, self.off_dev))
        self.t = t0  # capture ran no step
        if self.rate is not None:
            self.rate.t = t0
        torch.cuda.current_stream(dev).wait_stream(side)

    def step_graph(self):
        """One training step by replaying the captured graphs. Every check_every steps the pair-list
        status is read between the forward and the rest: an overflow grows the workspace,
        recaptures and redoes the forward before any gradient is taken."""
        self.g_fwd.replay()
        if self.t % self.check_every == 0:
            ok, needed = self.ws.status()
            if not ok:
                self.ws.allocate(int(needed * 1.15) + 1024)
                self._forward(True)
                self.capture()
        self.g_rest.replay()
        self.t += 1
        if self.rate is not None:
            self.rate.t = self.t

    def histogram_rate(self):
        """Histogram bits per attribute of the current attributes (float64 numpy)."""
        A = self.p.shape[0] - 3
        hb = histogram_bits(self.p[3:3 + A], 1.0 / 64)
        torch.cuda.synchronize()
        return hb.cpu().numpy()

    def eval_models(self):
        """Bits per attribute (float64 numpy) of the current attributes, symbols rint(y/q): the
        learned rate in evaluation mode, the empirical histogram (the judge), and the paper's own
        entropy models in evaluation mode (Sec. 3.3: the KDE of keyframe attributes and the Gaussian
        of residual attributes, each fitted per layer)."""
        from .entropy import GAUSSIAN, KDE, EntropyModel
        mlp, hist = self.eval_rate()
        A = self.p.shape[0] - 3
        out = {"mlp": mlp, "hist": hist}
        for name, kind in (("kde", KDE), ("gaussian", GAUSSIAN)):
            em = EntropyModel(A, self.n, kind, self.p.device, 1.0 / 64, self.levels, self.level_w, 1.0)
            out[name] = em.run(self.p[3:3 + A], 0).cpu().numpy()
            del em
        return out

    def eval_rate(self):
        """(MLP bits per attribute in evaluation mode, histogram bits per attribute), float64 numpy."""
        n = self.n
        A = self.rate.n_attr
        self.rate.reset()
        context(self.p, self.extent, self.levels, self.ctx)
        self.rate.run(_off(self.p, 3 * n), n, self.ctx, 0, self.levels, self.level_w, self.lam, grads=False)
        attrs = self.p[3:3 + A]
        hb = histogram_bits(attrs, self.rate.step_size)
        torch.cuda.synchronize()
        return self.rate.bits.cpu().numpy(), hb.cpu().numpy()


class RigidTrainer:
    """Rigid-transformation phase of inter-frame training (Sec. 3.2 rigid transformation, trained
    with the colour loss as in Sec. 3.3): the motion module predicts every Gaussian's translation and
    rotation from the previous frame's positions (the keyframe's means here), the frame is the
    keyframe composed with them (residual channels 0..6; the opacity residual stays 0), and the
    layer-weighted L1 against the frame's views trains the hash table and the MLP weights (Adam).

    One step, every compute step a C-ABI call: motion forward -> render forward (composition,
    projection, binning, rasterisation of all views and layers) -> fused L1 backward down to the
    residuals -> motion backward to the table and weights -> Adam on both."""

    def __init__(self, keyframe: torch.Tensor, cams: torch.Tensor, targets: torch.Tensor, settings: RenderSettings,
                 box_lo, box_hi, table: torch.Tensor, weights: torch.Tensor, lr_table: float = 1e-2,
                 lr_mlp: float = 1e-3, check_every: int = 1):
        from .motion import MotionModule
        dev = keyframe.device
        self.p, self.cams, self.tgt = keyframe, cams, targets
        self.n = keyframe.shape[1]
        self.st = dataclasses.replace(settings, res_channels=8)
        self.res = torch.zeros((1, 8, self.n), dtype=torch.float32, device=dev)
        self.d_res = torch.zeros_like(self.res)
        self.dp = torch.zeros_like(keyframe)  # the keyframe stays fixed in this phase
        self.table, self.weights = table, weights
        self.d_table, self.d_w = torch.zeros_like(table), torch.zeros_like(weights)
        self.opt_t, self.opt_w = Adam(table), Adam(weights)
        self.lr_table, self.lr_mlp = lr_table, lr_mlp
        self.mm = MotionModule(self.n, box_lo, box_hi, dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.t = 0
        self.check_every = max(1, int(check_every))  # pair-list status cadence, as in JointTrainer
        self.mm.forward(self.p, self.table, self.weights, self.res[0])
        self.img, self.ws = render_forward(self.st, self.p, cams, 1, self.res)  # sizes the workspace

    def step(self, check_overflow: bool | None = None):
        zero(self.loss)
        if check_overflow is None:
            check_overflow = self.t % self.check_every == 0
        self.mm.forward(self.p, self.table, self.weights, self.res[0])
        render_forward(self.st, self.p, self.cams, 1, self.res, ws=self.ws, image=self.img,
                       check_overflow=check_overflow)
        zero(self.d_res)
        zero(self.dp)
        render_backward(self.st, self.p, self.cams, self.ws, 1, self.res, image=self.img, target=self.tgt,
                        d_params=self.dp, d_residuals=self.d_res, loss=self.loss)
        self.mm.backward(self.p, self.table, self.weights, self.d_res[0], self.d_table, self.d_w)
        self.t += 1
        self.opt_t.step(self.d_table, self.lr_table, self.t)
        self.opt_w.step(self.d_w, self.lr_mlp, self.t)

    def translation(self) -> torch.Tensor:
        """The current predicted translation of every Gaussian, [3][n]."""
        return self.res[0, 0:3]


class ResidualTrainer:
    """Residual-deformation phase of inter-frame training (Sec. 3.2 residual deformation, trained with
    the inter-frame objective of Sec. 3.3): with the frame's translation and rotation fixed (rows
    0..6 of its residual block, e.g. from the rigid phase), the opacity, scale and colour residuals
    (rows 7..C-1) are trained with sum_l lambda^l (L1^l + lambda_rate R^l + lambda_reg |residuals|^l),
    R the Gaussian rate of the residual symbols (the paper's entropy model for residuals) and the
    last term the temporal L1.

    One step: render forward of all views and layers with the residuals -> fused L1 backward down
    to the residuals -> Gaussian rate + temporal L1 of the residual rows (their gradient added to
    the same rows) -> Adam on the residual rows."""

    def __init__(self, keyframe: torch.Tensor, residuals: torch.Tensor, cams: torch.Tensor, targets: torch.Tensor,
                 settings: RenderSettings, lambda_rate: float = 1e-4, lambda_reg: float = 1e-3, lr: float = 1e-3,
                 seed: int = 0, check_every: int = 1):
        from .entropy import GAUSSIAN, EntropyModel
        dev = keyframe.device
        C, n = keyframe.shape
        if tuple(residuals.shape) != (1, C, n):
            raise ValueError("residuals must be one frame's full block [1][C][n]")
        self.p, self.res, self.cams, self.tgt = keyframe, residuals, cams, targets
        self.n, self.C = n, C
        self.st = dataclasses.replace(settings, res_channels=C)
        self.d_res = torch.zeros_like(residuals)
        self.dp = torch.zeros_like(keyframe)
        self.opt = Adam(residuals)
        self.lr, self.seed = lr, seed
        levels = list(settings.level_counts) if settings.level_counts else [n]
        weights = list(settings.level_weights) if settings.level_weights else [1.0] * len(levels)
        self.ent = EntropyModel(C - 7, n, GAUSSIAN, dev, 1.0 / 64, levels, weights, lambda_rate, lambda_reg)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        self.rate_loss = torch.zeros(1, dtype=torch.float64, device=dev)
        self.t = 0
        self.check_every = max(1, int(check_every))  # pair-list status cadence, as in JointTrainer
        self.img, self.ws = render_forward(self.st, keyframe, cams, 1, residuals)  # sizes the workspace

    def step(self, check_overflow: bool | None = None):
        zero(self.loss)
        zero(self.rate_loss)
        if check_overflow is None:
            check_overflow = self.t % self.check_every == 0
        render_forward(self.st, self.p, self.cams, 1, self.res, ws=self.ws, image=self.img,
                       check_overflow=check_overflow)
        zero(self.d_res)
        zero(self.dp)
        render_backward(self.st, self.p, self.cams, self.ws, 1, self.res, image=self.img, target=self.tgt,
                        d_params=self.dp, d_residuals=self.d_res, loss=self.loss)
        A = self.C - 7
        self.ent.run(self.res[0, 7:], 1, seed=self.seed, offset=self.t * A * self.n, loss=self.rate_loss,
                     d_attrs=self.d_res[0, 7:])
        self.t += 1
        self.opt.step(self.d_res, self.lr, self.t, start=7 * self.n, count=(self.C - 7) * self.n)
