"""Python binding of the significance order and the quantise-to-2D-maps entry points
(gs_significance_order, gs_maps_describe, gs_encode_maps, gs_decode_maps): argument marshalling
only; every step runs in the HIP kernels of libgs4d.so."""
from __future__ import annotations

import ctypes

import torch

from ._lib import GsMapsLayout, check, lib
from .render import _check_tensor, _ptr, _stream


def significance_order(params: torch.Tensor, lambda_psi: float = 1e5, with_psi: bool = False):
    """Rank -> Gaussian index (int32 [n]) by Psi descending, ties by lower index; and Psi per
    Gaussian when with_psi."""
    _check_tensor(params, "params")
    C, n = params.shape
    order = torch.empty(n, dtype=torch.int32, device=params.device)
    psi = torch.empty(n, dtype=torch.float32, device=params.device) if with_psi else None
    nb = ctypes.c_size_t()
    check(lib().gs_significance_workspace_size(n, ctypes.byref(nb)), "gs_significance_workspace_size")
    ws = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=params.device)
    check(lib().gs_significance_order(n, _ptr(params), C, float(lambda_psi), _ptr(order), _ptr(psi), _ptr(ws),
                                      ws.numel(), _stream(params.device)), "gs_significance_order")
    return (order, psi) if with_psi else order


def maps_layout(n_channels: int, level_counts) -> GsMapsLayout:
    lv = (ctypes.c_int32 * 8)(*[int(x) for x in level_counts])
    lo = GsMapsLayout()
    check(lib().gs_maps_describe(n_channels, len(level_counts), lv, ctypes.byref(lo)), "gs_maps_describe")
    return lo


def encode_maps(params: torch.Tensor, order: torch.Tensor, level_counts, with_seq: bool = False):
    """(layout, ranges [L][C][2] float32, maps uint8 [total_bytes], seq int32 [n] or None)."""
    _check_tensor(params, "params")
    _check_tensor(order, "order", shape=(params.shape[1],), dtype=torch.int32, device=params.device)
    C, n = params.shape
    if int(level_counts[-1]) != n:
        raise ValueError("the last level count must equal the number of Gaussians")
    lo = maps_layout(C, level_counts)
    dev = params.device
    ranges = torch.empty((len(level_counts), C, 2), dtype=torch.float32, device=dev)
    maps = torch.empty(lo.total_bytes, dtype=torch.uint8, device=dev)
    seq = torch.empty(n, dtype=torch.int32, device=dev) if with_seq else None
    nb = ctypes.c_size_t()
    check(lib().gs_encode_workspace_size(ctypes.byref(lo), ctypes.byref(nb)), "gs_encode_workspace_size")
    ws = torch.empty(nb.value, dtype=torch.uint8, device=dev)
    check(lib().gs_encode_maps(ctypes.byref(lo), _ptr(params), _ptr(order), _ptr(ranges), _ptr(maps), _ptr(seq),
                               _ptr(ws), ws.numel(), _stream(dev)), "gs_encode_maps")
    return lo, ranges, maps, seq


def decode_maps(lo: GsMapsLayout, maps: torch.Tensor, ranges: torch.Tensor) -> torch.Tensor:
    """Parameters [C][n] in map order (the set a client renders, with the same level counts)."""
    _check_tensor(maps, "maps", shape=(lo.total_bytes,), dtype=torch.uint8)
    _check_tensor(ranges, "ranges", shape=(lo.n_levels, lo.n_channels, 2), device=maps.device)
    n = lo.level_counts[lo.n_levels - 1]
    out = torch.empty((lo.n_channels, n), dtype=torch.float32, device=maps.device)
    check(lib().gs_decode_maps(ctypes.byref(lo), _ptr(maps), _ptr(ranges), _ptr(out), _stream(maps.device)),
          "gs_decode_maps")
    return out


def planes(lo: GsMapsLayout, maps: torch.Tensor):
    """Views of the maps buffer: planes[l][c] is [height][width], uint16 codes for channels 0..2
    (as int32 values) and uint8 for the others."""
    out = []
    for l in range(lo.n_levels):
        w, h, off = lo.width[l], lo.height[l], lo.offset[l]
        layer = []
        for c in range(lo.n_channels):
            if c < 3:
                b = maps[off + 2 * w * h * c: off + 2 * w * h * (c + 1)]
                lo16 = b[0::2].to(torch.int32)
                hi16 = b[1::2].to(torch.int32)
                layer.append((lo16 | (hi16 << 8)).view(h, w))
            else:
                o = off + 2 * w * h * 3 + w * h * (c - 3)
                layer.append(maps[o:o + w * h].view(h, w))
        out.append(layer)
    return out
