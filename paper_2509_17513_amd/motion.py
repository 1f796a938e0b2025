"""Python binding of the rigid-motion module (gs_motion_forward / gs_motion_backward): argument
marshalling only; every step runs in the HIP kernels of libgs4d.so."""
from __future__ import annotations

import ctypes

import torch

from ._lib import GsMotionDesc, check, lib
from .render import _ptr, _stream


def sizes():
    """(hash-table floats, MLP weight count)."""
    t, w = ctypes.c_int64(), ctypes.c_int64()
    check(lib().gs_motion_sizes(ctypes.byref(t), ctypes.byref(w)), "gs_motion_sizes")
    return t.value, w.value


def _rows(t: torch.Tensor, rows: int, n: int, name: str):
    """A CUDA float32 array whose first `rows` rows (stride t.stride(0), contiguous along n) hold the data."""
    if (not t.is_cuda or t.dtype != torch.float32 or t.dim() != 2 or t.shape[0] < rows or t.shape[1] != n
            or t.stride(1) != 1):
        raise ValueError(f"{name} must be a float32 CUDA array with >= {rows} rows of {n} contiguous values")
    return t.stride(0)


class MotionModule:
    """The hash-grid + MLP motion predictor of one frame transition, for n Gaussians in a box."""

    def __init__(self, n: int, box_lo, box_hi, device):
        d = GsMotionDesc()
        d.n = n
        for a in range(3):
            d.box_lo[a], d.box_hi[a] = float(box_lo[a]), float(box_hi[a])
        self.desc, self.n, self.device = d, n, device
        nb = ctypes.c_size_t()
        check(lib().gs_motion_workspace_size(n, ctypes.byref(nb)), "gs_motion_workspace_size")
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=device)

    def forward(self, means: torch.Tensor, table: torch.Tensor, weights: torch.Tensor, out: torch.Tensor):
        """Writes rows 0..6 of `out` (a frame's residual block): translation and rotation."""
        rs = _rows(means, 3, self.n, "means")
        if _rows(out, 7, self.n, "out") != rs:
            raise ValueError("means and out must share one row stride")
        check(lib().gs_motion_forward(ctypes.byref(self.desc), _ptr(means), rs, _ptr(table), _ptr(weights), _ptr(out),
                                      _stream(self.device)), "gs_motion_forward")
        return out

    def backward(self, means, table, weights, d_out, d_table, d_weights):
        """Adds the gradients of the table and weights given dL/d(rows 0..6 of the residuals)."""
        rs = _rows(means, 3, self.n, "means")
        if _rows(d_out, 7, self.n, "d_out") != rs:
            raise ValueError("means and d_out must share one row stride")
        check(lib().gs_motion_backward(ctypes.byref(self.desc), _ptr(means), rs, _ptr(table), _ptr(weights),
                                       _ptr(d_out), _ptr(d_table), _ptr(d_weights), _ptr(self.ws), self.ws.numel(),
                                       _stream(self.device)), "gs_motion_backward")
