"""Oracle of the rigid-motion module of inter-frame training (Sec. 3.2, rigid transformation:
hash-grid features of the previous frame's Gaussian positions, Eq. 5, fed to two lightweight
MLPs that predict each Gaussian's translation and rotation, Eq. 6).

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU-baseline leg; it shares
no code with the GPU path.

The paper names the pieces, not their sizes; readings (the multi-resolution hash encoding as
published by Mueller et al. 2022, which the streaming methods the paper builds on use):
  * positions are mapped to the unit cube by the scene box, p = clamp((mu - lo) / (hi - lo), 0, 1);
  * L_h = 16 levels of F = 2 features, T = 2^15 entries per level; level l has resolution
    N_l = floor(16 b^l) with b = (1024 / 16)^(1 / 15); the point x = p N_l lies in the cell with
    corner c = min(floor(x), N_l - 1) and is interpolated trilinearly from the cell's 8 corners;
    a corner (i, j, k) is the table entry i + j (N_l + 1) + k (N_l + 1)^2 when (N_l + 1)^3 <= T,
    else (i * 1 xor j * 2654435761 xor k * 805459861) mod T in 32-bit unsigned arithmetic;
  * the 32 features feed two MLPs with two hidden layers of 64 ReLU units each and a linear
    output: Phi_mu -> translation d_mu (3), Phi_R -> rotation as the quaternion
    (1 + o0, o1, o2, o3) (the identity at zero output; it multiplies the previous rotation,
    R_t = dR R_{t-1}, and is normalised where it is used);
  * weights of a layer [out][in] row-major, then its bias.
The module's output is the translation and rotation residual of each Gaussian (channels 0..6 of
a frame's residuals); its backward takes their gradients to the hash table and the weights.
"""
from __future__ import annotations

import math

import numpy as np

LEVELS = 16
FEATS = 2
LOG2_T = 15
T = 1 << LOG2_T
N_MIN = 16
N_MAX = 1024
HIDDEN = 64
IN = LEVELS * FEATS
PRIMES = (1, 2654435761, 805459861)


def resolutions():
    """N_l = floor(16 b^l) (with a 1e-9 margin, so that 16 b^15 = 1024 is not floored to 1023)."""
    b = math.exp((math.log(N_MAX) - math.log(N_MIN)) / (LEVELS - 1))
    return [int(math.floor(N_MIN * b ** l + 1e-9)) for l in range(LEVELS)]


def head_sizes(out):
    """Parameter counts of one MLP: W1 [64][32], b1, W2 [64][64], b2, W3 [out][64], b3."""
    return [(HIDDEN, IN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (out, HIDDEN), (out,)]


def n_weights():
    return sum(int(np.prod(s)) for out in (3, 4) for s in head_sizes(out))


def unpack(w):
    """The flat weight vector as [(W1, b1, W2, b2, W3, b3) of Phi_mu, of Phi_R]."""
    w = np.asarray(w, np.float64)
    heads, off = [], 0
    for out in (3, 4):
        parts = []
        for s in head_sizes(out):
            k = int(np.prod(s))
            parts.append(w[off:off + k].reshape(s))
            off += k
        heads.append(parts)
    return heads


def corner_index(i, j, k, N):
    """Table entry of integer corner (i, j, k) at resolution N (arrays of int64)."""
    if (N + 1) ** 3 <= T:
        return i + j * (N + 1) + k * (N + 1) ** 2
    h = (np.asarray(i, np.uint64) * np.uint64(PRIMES[0])) & np.uint64(0xFFFFFFFF)
    h ^= (np.asarray(j, np.uint64) * np.uint64(PRIMES[1])) & np.uint64(0xFFFFFFFF)
    h ^= (np.asarray(k, np.uint64) * np.uint64(PRIMES[2])) & np.uint64(0xFFFFFFFF)
    return (h % np.uint64(T)).astype(np.int64)


def encode(means, lo, hi, table):
    """Features [n][32] and, per level, the corner entries [n][8] and weights [n][8]."""
    mu = np.asarray(means, np.float64).T  # [n][3]
    lo, hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
    p = np.clip((mu - lo) / (hi - lo), 0.0, 1.0)
    table = np.asarray(table, np.float64).reshape(LEVELS, T, FEATS)
    n = mu.shape[0]
    h = np.zeros((n, IN))
    corners = []
    for l, N in enumerate(resolutions()):
        x = p * N
        c = np.minimum(np.floor(x), N - 1).astype(np.int64)
        f = x - c
        idx = np.zeros((n, 8), np.int64)
        wts = np.zeros((n, 8))
        for k in range(8):
            di, dj, dk = k & 1, (k >> 1) & 1, (k >> 2) & 1
            idx[:, k] = corner_index(c[:, 0] + di, c[:, 1] + dj, c[:, 2] + dk, N)
            wts[:, k] = (np.where(di, f[:, 0], 1 - f[:, 0]) * np.where(dj, f[:, 1], 1 - f[:, 1]) *
                         np.where(dk, f[:, 2], 1 - f[:, 2]))
        h[:, FEATS * l:FEATS * (l + 1)] = np.einsum("nk,nkf->nf", wts, table[l][idx])
        corners.append((idx, wts))
    return h, corners


def _head_forward(h, W1, b1, W2, b2, W3, b3):
    z1 = h @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    return z1, a1, z2, a2, a2 @ W3.T + b3


def forward(means, lo, hi, table, weights):
    """Residual channels [7][n]: d_mu (3) and the rotation quaternion (4)."""
    h, _ = encode(means, lo, hi, table)
    (m1, m2) = unpack(weights)
    o_mu = _head_forward(h, *m1)[-1]
    o_r = _head_forward(h, *m2)[-1]
    q = o_r.copy()
    q[:, 0] += 1.0
    return np.concatenate([o_mu, q], axis=1).T


def min_preactivation(means, lo, hi, table, weights):
    """Per Gaussian, the smallest |pre-activation| of any hidden unit of either MLP: how close its
    ReLU decisions are to the kink (FP32 and FP64 can take the other side there)."""
    h, _ = encode(means, lo, hi, table)
    out = np.full(h.shape[0], np.inf)
    for head in unpack(weights):
        z1, _, z2, _, _ = _head_forward(h, *head)
        out = np.minimum(out, np.minimum(np.abs(z1).min(axis=1), np.abs(z2).min(axis=1)))
    return out


def backward(means, lo, hi, table, weights, d_out):
    """(d_table [16 * 2^15 * 2], d_weights [n_weights]) of the loss whose gradient in the
    module's output is d_out [7][n]."""
    h, corners = encode(means, lo, hi, table)
    heads = unpack(weights)
    d_out = np.asarray(d_out, np.float64).T  # [n][7]
    d_h = np.zeros_like(h)
    grads = []
    for (W1, b1, W2, b2, W3, b3), dy in zip(heads, (d_out[:, 0:3], d_out[:, 3:7])):
        z1, a1, z2, a2, _ = _head_forward(h, W1, b1, W2, b2, W3, b3)
        dz2 = (dy @ W3) * (z2 > 0)
        dz1 = (dz2 @ W2) * (z1 > 0)
        d_h += dz1 @ W1
        grads += [dz1.T @ h, dz1.sum(0), dz2.T @ a1, dz2.sum(0), dy.T @ a2, dy.sum(0)]
    d_table = np.zeros((LEVELS, T, FEATS))
    for l, (idx, wts) in enumerate(corners):
        for k in range(8):
            np.add.at(d_table[l], idx[:, k], wts[:, k:k + 1] * d_h[:, FEATS * l:FEATS * (l + 1)])
    return d_table.ravel(), np.concatenate([g.ravel() for g in grads])
