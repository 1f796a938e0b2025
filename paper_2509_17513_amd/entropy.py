"""Python binding of the paper's entropy models (gs_entropy_model): the KDE rate of keyframe
attributes (kind 0) and the Gaussian rate with the temporal L1 term of residual attributes
(kind 1). Argument marshalling only; every step runs in the HIP kernels of libgs4d.so."""
from __future__ import annotations

import ctypes

import torch

from ._lib import GsEntropyDesc, check, lib
from .render import _check_tensor, _ptr, _stream

KDE = 0
GAUSSIAN = 1


class EntropyModel:
    """The entropy model of one attribute set [A][n] with fixed layers; holds its workspace."""

    def __init__(self, n_attr: int, n: int, kind: int, device, step: float = 1.0 / 64, level_counts=None,
                 level_weights=None, lambda_rate: float = 1.0, lambda_reg: float = 0.0):
        lv = list(level_counts) if level_counts else [n]
        lw = list(level_weights) if level_weights else [1.0] * len(lv)
        if len(lv) > 8 or len(lw) != len(lv):
            raise ValueError("1..8 levels with one weight each")
        d = GsEntropyDesc()
        d.n, d.n_attr, d.step, d.kind = n, n_attr, step, kind
        d.n_levels = len(lv)
        for i in range(len(lv)):
            d.level_counts[i] = int(lv[i])
            d.level_weights[i] = float(lw[i])
        d.lambda_rate, d.lambda_reg = lambda_rate, lambda_reg
        self.desc, self.device = d, device
        nb = ctypes.c_size_t()
        check(lib().gs_entropy_workspace_size(ctypes.byref(d), ctypes.byref(nb)), "gs_entropy_workspace_size")
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=device)
        self.bits = torch.zeros(n_attr, dtype=torch.float64, device=device)

    def run(self, attrs: torch.Tensor, mode: int = 0, seed: int = 0, offset: int = 0, loss: torch.Tensor | None = None,
            sym_bits: torch.Tensor | None = None, d_attrs: torch.Tensor | None = None) -> torch.Tensor:
        """Per-attribute bits [A] (float64); adds L to `loss` (float64, one element), writes the
        per-symbol bits and adds dL/dy to `d_attrs` (mode 1) when given."""
        d = self.desc
        _check_tensor(attrs, "attrs", shape=(d.n_attr, d.n), device=self.device)
        _check_tensor(loss, "loss", shape=(1,), dtype=torch.float64, device=self.device)
        _check_tensor(sym_bits, "sym_bits", shape=(d.n_attr, d.n), device=self.device)
        _check_tensor(d_attrs, "d_attrs", shape=(d.n_attr, d.n), device=self.device)
        d.mode, d.seed, d.offset = mode, seed, offset
        check(lib().gs_entropy_model(ctypes.byref(d), _ptr(attrs), _ptr(self.bits), _ptr(loss), _ptr(sym_bits),
                                     _ptr(d_attrs), _ptr(self.ws), self.ws.numel(), _stream(self.device)),
              "gs_entropy_model")
        return self.bits
