"""Oracle of the significance ordering and the quantise-to-2D-maps step of the progressive
bitstream (Sec. 3.1, significance metric; Sec. 3.3, progressive bitstream generation; App. A).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU-baseline leg; it shares
no code with the GPU path.

Readings (the paper states the metric and the bit depths, not the layout):
  * significance Psi_i = opacity_i + lambda_psi * (4/3) pi a_i b_i c_i, with opacity = sigmoid of
    the stored logit and a, b, c = exp of the stored log-scales; Gaussians are ranked by Psi
    descending, ties by lower index, and layer l holds ranks [N_{l-1}, N_l);
  * per layer and channel, the values are quantised with that layer's minimum and maximum:
    code = rint((v - min) * ((2^b - 1) / (max - min))) (half to even; code 0 when max == min),
    b = 16 for the three position channels, 8 for every other channel; decoding is
    min + code * ((max - min) / (2^b - 1));
  * each channel of a layer is one 2D map: the layer's Gaussians are ordered by the Morton code of
    their position codes (top 10 bits of x and y, top 9 of z, interleaved x, y, z from the least
    significant bit; ties by rank) and written 256 at a time into 16 x 16 blocks, the blocks
    snaking row by row (even block rows left to right, odd ones right to left) and the 256
    Gaussians of a block along the 2D Morton curve inside it (x bit first); the map is
    W = 16 ceil(ceil(sqrt(m)) / 16) wide and H = 16 ceil(ceil(m / W) / 16) tall, and pixels past
    the layer's m Gaussians repeat its last Gaussian.
The quantisation codes are integer decisions taken in FP32 on both sides (the same operations in
the same order); everything else is exact integer arithmetic.
"""
from __future__ import annotations

import numpy as np

POS_BITS = 16
ATTR_BITS = 8


def significance(params, lambda_psi: float = 1e5) -> np.ndarray:
    """Psi of every Gaussian in FP64. params [C][n] (0..2 mean, 3..5 log-scale, 10 opacity logit)."""
    p = np.asarray(params, np.float64)
    opacity = 1.0 / (1.0 + np.exp(-p[10]))
    volume = 4.0 / 3.0 * np.pi * np.exp(p[3]) * np.exp(p[4]) * np.exp(p[5])
    return opacity + lambda_psi * volume


def significance_order(params, lambda_psi: float = 1e5) -> np.ndarray:
    """Rank -> Gaussian index: Psi descending, ties by lower index."""
    psi = significance(params, lambda_psi)
    idx = np.arange(psi.size)
    return np.lexsort((idx, -psi)).astype(np.int64)


def channel_bits(c: int) -> int:
    return POS_BITS if c < 3 else ATTR_BITS


def quantise(v, mn, mx, bits: int) -> np.ndarray:
    """FP32 codes of values v with the range [mn, mx] (see the module readings)."""
    v = np.asarray(v, np.float32)
    mn, mx = np.float32(mn), np.float32(mx)
    top = np.float32(2 ** bits - 1)
    if not mx > mn:
        return np.zeros(v.shape, np.int64)
    scale = np.float32(top / np.float32(mx - mn))
    code = np.rint(np.float32(v - mn) * scale)
    return np.clip(code, 0, 2 ** bits - 1).astype(np.int64)


def dequantise(code, mn, mx, bits: int) -> np.ndarray:
    """FP64 value of codes (the GPU rounds the same expression once, in FP32)."""
    step = (float(mx) - float(mn)) / (2 ** bits - 1)
    return float(mn) + np.asarray(code, np.float64) * step


def morton3(x, y, z) -> np.ndarray:
    """Interleave bits: x bit k -> 3k, y bit k -> 3k+1, z bit k -> 3k+2 (x, y 10 bits, z 9)."""
    x, y, z = (np.asarray(a, np.int64) for a in (x, y, z))
    out = np.zeros(x.shape, np.int64)
    for k in range(10):
        out |= ((x >> k) & 1) << (3 * k)
        out |= ((y >> k) & 1) << (3 * k + 1)
        if k < 9:
            out |= ((z >> k) & 1) << (3 * k + 2)
    return out


def map_size(m: int):
    w = 16 * -(-int(np.ceil(np.sqrt(m))) // 16) if m > 0 else 16
    h = 16 * -(-(-(-m // w)) // 16) if m > 0 else 16
    return w, h


def block_pixel(p, w: int):
    """Pixel (x, y) of sequence position(s) p of a layer whose map is w wide."""
    p = np.asarray(p, np.int64)
    blk, q = p // 256, p % 256
    nbx = w // 16
    by, bx = blk // nbx, blk % nbx
    bx = np.where(by % 2 == 1, nbx - 1 - bx, bx)
    u = np.zeros_like(q)
    v = np.zeros_like(q)
    for k in range(4):
        u |= ((q >> (2 * k)) & 1) << k
        v |= ((q >> (2 * k + 1)) & 1) << k
    return 16 * bx + u, 16 * by + v


def encode(params, order, level_counts):
    """Layer ranges [L][C][2] (min, max) and maps: a list over layers of [C][H][W] int64 codes,
    plus for every layer the Gaussian index of each of its m sequence positions."""
    p = np.asarray(params, np.float32)
    C, n = p.shape
    order = np.asarray(order, np.int64)
    lv = [0] + list(level_counts)
    ranges = np.zeros((len(level_counts), C, 2), np.float32)
    maps, seqs = [], []
    for l in range(len(level_counts)):
        idx = order[lv[l]:lv[l + 1]]
        m = idx.size
        vals = p[:, idx]
        if m > 0:
            ranges[l, :, 0] = vals.min(axis=1)
            ranges[l, :, 1] = vals.max(axis=1)
        codes = np.stack([quantise(vals[c], ranges[l, c, 0], ranges[l, c, 1], channel_bits(c)) for c in range(C)]) \
            if m > 0 else np.zeros((C, 0), np.int64)
        if m > 0:
            key = morton3(codes[0] >> 6, codes[1] >> 6, codes[2] >> 7)
            seq = np.lexsort((np.arange(m), key))  # Morton ascending, ties by rank
        else:
            seq = np.zeros(0, np.int64)
        w, h = map_size(m)
        mp = np.zeros((C, h, w), np.int64)
        if m > 0:
            pos = np.arange(w * h)
            x, y = block_pixel(pos, w)
            mp[:, y, x] = codes[:, seq[np.minimum(pos, m - 1)]]
        maps.append(mp)
        seqs.append(idx[seq])
    return ranges, maps, seqs


def decode(ranges, maps, level_counts):
    """FP64 parameters [C][n] in map order (layer by layer, sequence position by position)."""
    C = maps[0].shape[0]
    lv = [0] + list(level_counts)
    out = np.zeros((C, lv[-1]), np.float64)
    for l in range(len(level_counts)):
        m = lv[l + 1] - lv[l]
        x, y = block_pixel(np.arange(m), maps[l].shape[2])
        for c in range(C):
            out[c, lv[l]:lv[l + 1]] = dequantise(maps[l][c, y, x], ranges[l, c, 0], ranges[l, c, 1], channel_bits(c))
    return out
