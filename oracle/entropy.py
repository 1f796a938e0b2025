"""Oracle of the paper's own entropy models of the quantised attributes (Sec. 3.3): the KDE rate of
keyframe attributes and the Gaussian rate and temporal L1 term of residual attributes.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and the benchmark's CPU-baseline leg; it shares
no code with the GPU path (the noise generator and the layer weights come from ``oracle.rate``).

Symbols: attribute a of Gaussian i is y; mode 0 evaluates the quantised value rint(y / q) q,
mode 1 the noisy one y + u q with u uniform in [-1/2, 1/2) from the counter-based SplitMix64
generator of ``oracle.rate.noise``. The density of a symbol is estimated from the symbols of the
same attribute in the same layer (Sec. 3.3: the entropy of a level is estimated from that level's
attributes), and a symbol costs bits = -log2 max(P, 1e-9) with P = F(y + q/2) - F(y - q/2) for
the estimated CDF F (the PMF as CDF differences).

KDE (keyframe attributes), in the paper's order of steps:
  1. Silverman's rule: h = sigma (3 m / 4)^(-1/5) with sigma the sample standard deviation
     (m - 1 in the denominator) of the layer's m symbols, as scipy's gaussian_kde uses it; h is
     at least q / 4 (a layer of equal symbols);
  2. the CDF on a grid through a convolution: the symbols are linearly binned on the grid
     x_k = lo + k Delta (Delta = min(q, h) / 4, lo = min - 8 h - q, up to max + 8 h + q; Delta is
     widened if the grid would pass 16384 points or the kernel 3071 points a side), and the
     binned counts are convolved (FFT) with the kernel's CDF, F_k = sum_j c_j Phi((k - j) Delta / h) / m;
  3. the PMF by differencing the CDF one step apart, the CDF taken between grid points by linear
     interpolation.
  The binned density is held fixed for the gradient (binning has no derivative): dbits/dy comes
  from the slopes of the interpolated CDF at y +- q/2.
Gaussian (residual attributes): F is the normal CDF with the layer's symbol mean mu and standard
  deviation sigma = max(sqrt(mean((y - mu)^2)), q 1e-3); the gradient includes the dependence of
  mu and sigma on every symbol. The temporal term adds lambda_reg |y| per symbol.
Loss: L = sum_i w_i bits_i (+ sum_i lambda^l lambda_reg |y_i| for the residual model), with
  w_i = lambda_rate lambda^l / |G^l| (the per-level rate of Sec. 3.3 weighted by lambda^l).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

from . import rate

P_FLOOR = 1e-9
G_MAX = 16384
K_MAX = 3071
LN2 = math.log(2.0)


def symbols(attrs, step, mode, seed=0, offset=0):
    """[A][n] FP64 symbols (mode 0 quantised, mode 1 noisy; FP32 arithmetic like the attributes)."""
    y = np.asarray(attrs, np.float32)
    if mode == 0:
        q = np.float32(step)
        return (np.rint(y / q) * q).astype(np.float32).astype(np.float64)
    A, n = y.shape
    u = rate.noise(A, n, step, seed, offset)  # u q, already scaled, FP32 values
    return (y + u.astype(np.float32)).astype(np.float32).astype(np.float64)


def silverman(y, step):
    m = y.size
    sigma = float(np.std(y, ddof=1)) if m > 1 else 0.0
    return max(sigma * (3.0 * m / 4.0) ** (-0.2), step / 4.0)


def kde_grid(y, step):
    """(h, lo, Delta, G, K) of the KDE of the symbols y of one layer and attribute."""
    h = silverman(y, step)
    pad = 8.0 * h + step
    lo, hi = float(y.min()) - pad, float(y.max()) + pad
    delta = max(min(step, h) / 4.0, (hi - lo) / (G_MAX - 1), 8.0 * h / K_MAX)
    G = int(math.ceil((hi - lo) / delta)) + 1
    K = int(math.ceil(8.0 * h / delta))
    return h, lo, delta, G, K


def kde_cdf(y, step):
    """Grid CDF F[G] (FP64) and the grid (h, lo, Delta, G, K) of one layer's symbols."""
    h, lo, delta, G, K = kde_grid(y, step)
    t = (y - lo) / delta
    k = np.floor(t).astype(np.int64)
    f = t - k
    c = np.zeros(G + 1)
    np.add.at(c, k, 1.0 - f)
    np.add.at(c, k + 1, f)
    c = c[:G]
    # F_k = sum_j c_j Phi((k - j) Delta / h) / m: a linear convolution of c with the kernel's CDF
    # sampled at every offset d = k - j in [-(G - 1), G - 1], by FFT
    d = np.arange(-(G - 1), G)
    ker = 0.5 * erfc(-(d * delta / h) / math.sqrt(2.0))
    size = 1 << int(math.ceil(math.log2(3 * G)))
    conv = np.fft.irfft(np.fft.rfft(c, size) * np.fft.rfft(ker, size), size)
    F = conv[G - 1:2 * G - 1] / y.size
    return F, (h, lo, delta, G, K)


def _interp(F, lo, delta, x):
    G = F.size
    t = (x - lo) / delta
    k = np.clip(np.floor(t).astype(np.int64), 0, G - 2)
    f = t - k
    val = F[k] + f * (F[k + 1] - F[k])
    slope = (F[k + 1] - F[k]) / delta
    return val, slope


def kde_bits(y, step):
    """Per symbol (bits, dbits/dy with the density held fixed) of one layer's symbols y."""
    F, (h, lo, delta, G, K) = kde_cdf(y, step)
    Fp, sp = _interp(F, lo, delta, y + step / 2)
    Fm, sm = _interp(F, lo, delta, y - step / 2)
    P = Fp - Fm
    floored = P < P_FLOOR
    bits = -np.log2(np.maximum(P, P_FLOOR))
    dbits = np.where(floored, 0.0, -(sp - sm) / (np.maximum(P, P_FLOOR) * LN2))
    return bits, dbits


def gaussian_bits(y, step):
    """Per symbol (bits, total dbits_sum/dy_k) of one layer's symbols y under the Gaussian model,
    the gradient of sum_i bits_i including the dependence of mu and sigma on every symbol."""
    m = y.size
    mu = float(y.mean())
    sd = math.sqrt(float(np.mean((y - mu) ** 2)))
    sigma = max(sd, step * 1e-3)
    a = (y - mu + step / 2) / sigma
    b = (y - mu - step / 2) / sigma
    # P = Phi(a) - Phi(b), from the tail that keeps it accurate
    P = np.where(b > 0, 0.5 * (erfc(b / math.sqrt(2)) - erfc(a / math.sqrt(2))),
                 0.5 * (erfc(-a / math.sqrt(2)) - erfc(-b / math.sqrt(2))))
    floored = P < P_FLOOR
    Pc = np.maximum(P, P_FLOOR)
    bits = -np.log2(Pc)
    pa, pb = np.exp(-0.5 * a * a) / math.sqrt(2 * math.pi), np.exp(-0.5 * b * b) / math.sqrt(2 * math.pi)
    dP_dy = (pa - pb) / sigma
    dP_dsig = -(a * pa - b * pb) / sigma
    g = np.where(floored, 0.0, -1.0 / (Pc * LN2))  # dbits/dP
    d_y = g * dP_dy
    d_mu = -d_y
    d_sig = g * dP_dsig
    # mu = mean(y), sigma = sqrt(mean((y - mu)^2)) (when not at its floor)
    total = d_y + d_mu.sum() / m
    if sd > step * 1e-3:
        total = total + d_sig.sum() * (y - mu) / (m * sd)
    return bits, total, d_y


def entropy_model(attrs, step, kind, mode=0, seed=0, offset=0, level_counts=None, level_weights=None,
                  lambda_rate=1.0, lambda_reg=0.0):
    """(bits per attribute [A], loss, per-symbol bits [A][n], dL/dy [A][n]) for kind 0 (KDE) or
    1 (Gaussian + temporal L1)."""
    attrs = np.asarray(attrs, np.float32)
    A, n = attrs.shape
    lv = list(level_counts) if level_counts else [n]
    lw = list(level_weights) if level_weights else [1.0] * len(lv)
    y = symbols(attrs, step, mode, seed, offset)
    sym = np.zeros((A, n))
    grad = np.zeros((A, n))
    loss = 0.0
    bounds = [0] + lv
    for l in range(len(lv)):
        s0, s1 = bounds[l], bounds[l + 1]
        m = s1 - s0
        if m == 0:
            continue
        w = lambda_rate * lw[l] / m
        for a in range(A):
            ya = y[a, s0:s1]
            if kind == 0:
                bits, db = kde_bits(ya, step)
                g = w * db
            else:
                bits, total, _ = gaussian_bits(ya, step)
                g = w * total + lw[l] * lambda_reg * np.sign(ya)
                loss += lw[l] * lambda_reg * np.abs(ya).sum()
            sym[a, s0:s1] = bits
            grad[a, s0:s1] = g
            loss += w * bits.sum()
    return sym.sum(axis=1), loss, sym, grad
