"""FP64 oracle of the rate terms of the quantised Gaussian attributes.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Symbols: an attribute y quantised with step q has symbol k = rint(y / q)
  (round half to even); the paper simulates quantisation in training with
  additive uniform noise of one step's width (Sec. 3.3, differentiable
  quantisation; the noise here is u ~ U(-q/2, q/2)).
* Histogram rate (the reference of the learned rate): bits = -sum_i log2(n(k_i) / N) over the
  empirical symbol counts n(k) of one attribute, i.e. N times the empirical
  entropy.
* Learned rate: a discretised Laplace per symbol, PMF(y) = F(y + q/2) - F(y - q/2)
  (the PMF of Sec. 3.3 written in value units, one step wide), whose location
  m and scale b come from a small per-attribute MLP of a 16-feature context of
  the Gaussian: 16 -> 64 -> 64 -> 2 with tanh-GELU, BF16 weights and
  activations, FP32 biases; m = out0, b = softplus(out1) + q / 16. The rate
  is -log2(max(PMF, 1e-9)).
* Noise: the counter-based SplitMix64 generator (Steele, Lea & Flood 2014):
  z = seed + (offset + a * n + i + 1) * 0x9E3779B97F4A7C15 (mod 2^64), then the
  SplitMix64 output mix; u = (z >> 40) * 2^-24 - 0.5, noise = u * q.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
P_FLOOR = 1e-9
CTX_DIM, HIDDEN = 16, 64
W1_OFF, W2_OFF, W3_OFF = 0, 16 * 64, 16 * 64 + 64 * 64
W_PER_ATTR = 16 * 64 + 64 * 64 + 2 * 64   # BF16 matrix weights per attribute
B1_OFF, B2_OFF, B3_OFF = 0, 64, 128
B_PER_ATTR = 64 + 64 + 2                  # FP32 biases per attribute


# ------------------------------------------------------------------ BF16
def bf16_round(x):
    """Round float64 values to the nearest BF16 (ties to even), returned as float64.
    Written on the bit pattern of the float32 nearest to x after exact FP64 rounding:
    first to float32 would double-round, so it works from float64 directly."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)  # x = m * 2^e, 0.5 <= |m| < 1
    # BF16 keeps 8 significant bits: scale so the kept bits are the integer part
    scaled = np.ldexp(m, 8)
    r = np.rint(scaled)  # numpy rint = round half to even
    out = np.ldexp(r, e - 8)
    return np.where(np.isfinite(x), out, x)


def bf16_bits_to_f64(u16):
    u = np.asarray(u16, np.uint32) << np.uint32(16)
    return u.view(np.float32).astype(np.float64)


def f64_to_bf16_bits(x):
    r = bf16_round(x).astype(np.float32)
    return (r.view(np.uint32) >> np.uint32(16)).astype(np.uint16)


# ---------------------------------------------------------- SplitMix64 noise
def splitmix64(z):
    z = np.asarray(z, np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def noise(n_attr, n, step, seed, offset):
    """[n_attr][n] uniform noise in [-step/2, step/2)."""
    a = np.arange(n_attr, dtype=np.uint64)[:, None]
    i = np.arange(n, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        ctr = np.uint64(offset) + a * np.uint64(n) + i + np.uint64(1)
        z = np.uint64(seed) + ctr * GOLDEN
    u = (splitmix64(z) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24 - 0.5
    return (u * np.float32(step)).astype(np.float32).astype(np.float64)


# --------------------------------------------------------- discretised Laplace
def laplace_bits(y, m, b, step):
    """-log2 max(F(y + q/2) - F(y - q/2), 1e-9) for the Laplace(m, b) CDF F, elementwise.
    Returns (bits, dbits/dy, dbits/db); dbits/dm = -dbits/dy. Gradients are 0 where the floor binds."""
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        return _laplace_bits(y, m, b, step)


def _laplace_bits(y, m, b, step):
    y, m, b = (np.asarray(v, np.float64) for v in (y, m, b))
    h = 0.5 * step
    d = y - m
    t = np.abs(d)
    sg = np.sign(d)
    far = t >= h
    # t >= h: P = 1/2 exp(-(t - h)/b) (1 - exp(-q/b))
    lp_far = math.log(0.5) - (t - h) / b + np.log(-np.expm1(-step / b))
    dlp_dt_far = -1.0 / b
    dlp_db_far = (t - h) / b ** 2 - (step / b ** 2) / np.expm1(step / b)
    # t < h: P = 1 - 1/2 exp(-(h + t)/b) - 1/2 exp(-(h - t)/b)
    ea = np.exp(-(h + t) / b)
    eb = np.exp(-(h - t) / b)
    P_near = 1.0 - 0.5 * ea - 0.5 * eb
    lp_near = np.log(np.maximum(P_near, 1e-300))
    dP_dt = 0.5 * ea / b - 0.5 * eb / b
    dP_db = -0.5 * ea * (h + t) / b ** 2 - 0.5 * eb * (h - t) / b ** 2
    lp = np.where(far, lp_far, lp_near)
    dlp_dt = np.where(far, dlp_dt_far, dP_dt / np.maximum(P_near, 1e-300))
    dlp_db = np.where(far, dlp_db_far, dP_db / np.maximum(P_near, 1e-300))
    floored = lp < math.log(P_FLOOR)
    lp = np.maximum(lp, math.log(P_FLOOR))
    bits = -lp / math.log(2.0)
    dbits_dy = np.where(floored, 0.0, -dlp_dt * sg / math.log(2.0))
    dbits_db = np.where(floored, 0.0, -dlp_db / math.log(2.0))
    return bits, dbits_dy, dbits_db


def laplace_pmf(k, m, b, step):
    """PMF of symbol k (value k * step) written directly from the CDF (for pins)."""
    def F(x):
        z = (x - m) / b
        return np.where(z < 0, 0.5 * np.exp(z), 1.0 - 0.5 * np.exp(-z))
    y = np.asarray(k, np.float64) * step
    return F(y + step / 2) - F(y - step / 2)


# ------------------------------------------------------------ histogram rate
def hist_bits(attrs, step):
    """Per-attribute histogram rate in bits: -sum_i log2(n(k_i)/N), k = rint(y/q). attrs [A][N]."""
    attrs = np.asarray(attrs, np.float32)
    A, N = attrs.shape
    out = np.zeros(A)
    for a in range(A):
        k = np.rint(attrs[a].astype(np.float64) / np.float64(np.float32(step)))
        _, cnt = np.unique(k, return_counts=True)
        cnt = cnt.astype(np.float64)
        out[a] = -(cnt * np.log2(cnt / N)).sum()
    return out


def bucketed_hist_bits(attrs, step, bucket):
    """Histogram rate conditioned on a bucket per Gaussian (e.g. its layer x position octant):
    per attribute -sum_i log2(n(b_i, k_i) / N(b_i)), the empirical conditional entropy times N.
    It is the rate a coder that knows each Gaussian's bucket reaches with per-bucket histograms;
    with one bucket it is hist_bits. attrs [A][N], bucket [N] integer labels."""
    attrs = np.asarray(attrs, np.float32)
    bucket = np.asarray(bucket)
    A, N = attrs.shape
    out = np.zeros(A)
    _, bi = np.unique(bucket, return_inverse=True)
    nb = np.bincount(bi).astype(np.float64)
    for a in range(A):
        k = np.rint(attrs[a].astype(np.float64) / np.float64(np.float32(step)))
        _, ki = np.unique(k, return_inverse=True)
        _, cnt = np.unique(bi.astype(np.int64) * (ki.max() + 1) + ki, return_inverse=True)
        n_bk = np.bincount(cnt).astype(np.float64)[cnt]
        out[a] = -np.log2(n_bk / nb[bi]).sum()
    return out


def layer_octant_bucket(means, layer):
    """Bucket label of each Gaussian: its layer (1..L) times the octant of its mean (sign of x, y, z)."""
    m = np.asarray(means, np.float64)
    octant = (m[0] >= 0).astype(np.int64) + 2 * (m[1] >= 0) + 4 * (m[2] >= 0)
    return np.asarray(layer, np.int64) * 8 + octant


# ------------------------------------------------------------------- context
def context(means, extent, layer_of):
    """16 features per Gaussian: mean / extent (3), sin and cos of pi 2^k mean / extent for
    k = 0, 1 (12), (layer - 1) / 5 (1); rounded to BF16. means [3][N], layer_of [N] in 1..L."""
    u = np.asarray(means, np.float32).astype(np.float64) / np.float64(np.float32(extent))
    feats = [u]
    for k in range(2):
        feats.append(np.sin(math.pi * 2 ** k * u))
        feats.append(np.cos(math.pi * 2 ** k * u))
    feats.append(((np.asarray(layer_of, np.float64) - 1.0) / 5.0)[None])
    x = np.concatenate(feats, axis=0)  # [16][N]
    return bf16_round(x)


def layer_of(n, level_counts):
    lv = np.asarray(level_counts)
    return 1 + np.searchsorted(lv, np.arange(n), side="right")


def symbol_weights(n, level_counts, level_weights, lambda_rate):
    """w_i = lambda_rate * lambda^l / |G^l| for the layer l of Gaussian i."""
    lv = [0] + list(level_counts)
    w = np.zeros(n)
    for l in range(len(level_counts)):
        lo, hi = lv[l], lv[l + 1]
        if hi > lo:
            w[lo:hi] = lambda_rate * level_weights[l] / (hi - lo)
    return w


# ----------------------------------------------------------------------- MLP
def gelu(x):
    c = math.sqrt(2.0 / math.pi)
    return 0.5 * x * (1.0 + np.tanh(c * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    c = math.sqrt(2.0 / math.pi)
    u = c * (x + 0.044715 * x ** 3)
    th = np.tanh(u)
    return 0.5 * (1.0 + th) + 0.5 * x * (1.0 - th ** 2) * c * (1.0 + 3 * 0.044715 * x ** 2)


def softplus(x):
    return np.log1p(np.exp(-np.abs(x))) + np.maximum(x, 0.0)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def unpack(w_bf16_bits, b_f32, a, weights_f64=None):
    """Per-attribute (W1 [64][16], b1, W2 [64][64], b2, W3 [2][64], b3) as float64."""
    W = bf16_bits_to_f64(w_bf16_bits[a]) if weights_f64 is None else np.asarray(weights_f64[a], np.float64)
    B = np.asarray(b_f32[a], np.float64)
    return (W[W1_OFF:W2_OFF].reshape(64, 16), B[B1_OFF:B2_OFF], W[W2_OFF:W3_OFF].reshape(64, 64), B[B2_OFF:B3_OFF],
            W[W3_OFF:].reshape(2, 64), B[B3_OFF:])


def rate_model(attrs, ctx, w_bf16_bits, b_f32, step, mode=0, seed=0, offset=0, sym_w=None, emulate_bf16=True,
               want_grad=True, weights_f64=None, fit_scale=None, want_abs=False):
    """Learned rate. attrs [A][N] float32, ctx [16][N] (BF16 values as float64).
    Returns dict: bits [A] (unweighted per-attribute totals), loss (sum_i w_i sum_a bits),
    d_attrs [A][N] (train mode: dloss/dy through the additive noise), d_w [A][W_PER_ATTR],
    d_b [A][B_PER_ATTR] (gradients of fit_scale * sum_i sum_a bits, the maximum-likelihood fit of
    the entropy model; of the loss itself when fit_scale is None), m, b [A][N]; with want_abs also
    d_w_abs, d_b_abs: the same sums over symbols taken of the absolute values of their terms."""
    attrs = np.asarray(attrs, np.float32).astype(np.float64)
    A, N = attrs.shape
    q = float(np.float32(step))
    if mode == 0:
        yh = np.rint(attrs / q) * q
    else:
        yh = (attrs.astype(np.float32) + noise(A, N, step, seed, offset).astype(np.float32)).astype(np.float64)
    sym_w = np.ones(N) if sym_w is None else np.asarray(sym_w, np.float64)
    rnd = bf16_round if emulate_bf16 else (lambda v: v)
    X = np.asarray(ctx, np.float64).T  # [N][16]
    out = {"bits": np.zeros(A), "loss": 0.0, "d_attrs": np.zeros((A, N)), "d_w": np.zeros((A, W_PER_ATTR)),
           "d_b": np.zeros((A, B_PER_ATTR)), "m": np.zeros((A, N)), "b": np.zeros((A, N))}
    if want_abs:
        out["d_w_abs"] = np.zeros((A, W_PER_ATTR))
        out["d_b_abs"] = np.zeros((A, B_PER_ATTR))
    for a in range(A):
        W1, b1, W2, b2, W3, b3 = unpack(w_bf16_bits, b_f32, a, weights_f64)
        z1 = X @ W1.T + b1
        h1 = rnd(gelu(z1))
        z2 = h1 @ W2.T + b2
        h2 = rnd(gelu(z2))
        o = h2 @ W3.T + b3
        m = o[:, 0]
        sb = softplus(o[:, 1])
        bb = sb + q / 16.0
        bits, dy, dbb = laplace_bits(yh[a], m, bb, q)
        out["bits"][a] = bits.sum()
        out["loss"] += float((sym_w * bits).sum())
        out["m"][a], out["b"][a] = m, bb
        if not want_grad:
            continue
        g_y = sym_w * dy
        if mode == 1:
            out["d_attrs"][a] = g_y
        fw = sym_w if fit_scale is None else np.full(N, float(np.float32(fit_scale)))
        do = np.stack([-fw * dy, fw * dbb * sigmoid(o[:, 1])], axis=1)  # [N][2]
        dW3 = do.T @ h2
        dh2 = do @ W3
        dz2 = dh2 * gelu_grad(z2)
        dW2 = dz2.T @ h1
        dh1 = dz2 @ W2
        dz1 = dh1 * gelu_grad(z1)
        dW1 = dz1.T @ X
        out["d_w"][a] = np.concatenate([dW1.reshape(-1), dW2.reshape(-1), dW3.reshape(-1)])
        out["d_b"][a] = np.concatenate([dz1.sum(0), dz2.sum(0), do.sum(0)])
        if want_abs:
            ado, adz2, adz1 = np.abs(do), np.abs(dz2), np.abs(dz1)
            out["d_w_abs"][a] = np.concatenate([(adz1.T @ np.abs(X)).reshape(-1), (adz2.T @ np.abs(h1)).reshape(-1),
                                                (ado.T @ np.abs(h2)).reshape(-1)])
            out["d_b_abs"][a] = np.concatenate([adz1.sum(0), adz2.sum(0), ado.sum(0)])
    return out


def init_weights(n_attr, seed, attrs=None, step=1.0 / 64):
    """Seeded initial weights: W ~ N(0, 1/fan_in) as BF16 bits, biases 0 except the output bias,
    set from the attribute's mean and mean absolute deviation when attrs is given."""
    rng = np.random.default_rng(seed)
    W = np.zeros((n_attr, W_PER_ATTR))
    W[:, W1_OFF:W2_OFF] = rng.standard_normal((n_attr, 64 * 16)) / 4.0
    W[:, W2_OFF:W3_OFF] = rng.standard_normal((n_attr, 64 * 64)) / 8.0
    W[:, W3_OFF:] = rng.standard_normal((n_attr, 2 * 64)) / 8.0 * 0.1
    Bv = np.zeros((n_attr, B_PER_ATTR), np.float32)
    if attrs is not None:
        a64 = np.asarray(attrs, np.float64)
        mu = a64.mean(axis=1)
        mad = np.abs(a64 - mu[:, None]).mean(axis=1)
        Bv[:, B3_OFF] = mu
        target = np.maximum(mad - step / 16, step / 4)
        Bv[:, B3_OFF + 1] = np.log(np.expm1(target))  # softplus^-1
    return f64_to_bf16_bits(W), Bv


# ------------------------------------------------------- context-free baselines
def laplace_fit_bits(attrs, step):
    """Context-free baseline of the learned rate (the method without its context): per attribute a
    Laplace with the maximum-likelihood location (median) and scale (mean absolute deviation), bits
    of the rint-quantised symbols under its PMF (CDF differences one step apart, floor 1e-9)."""
    out = np.zeros(attrs.shape[0])
    for a in range(attrs.shape[0]):
        y = np.rint(attrs[a].astype(np.float64) / step) * step
        m = np.median(y)
        b = max(np.abs(y - m).mean(), step / 16)
        t = np.abs(y - m)
        h = step / 2
        with np.errstate(divide="ignore", over="ignore"):
            far = math.log(0.5) - (t - h) / b + math.log(-math.expm1(-step / b))
            near = np.log(np.maximum(1 - 0.5 * np.exp(-(h + t) / b) - 0.5 * np.exp(-(h - t) / b), 1e-300))
        lp = np.maximum(np.where(t >= h, far, near), math.log(1e-9))
        out[a] = -lp.sum() / math.log(2)
    return out


def gaussian_fit_bits(attrs, step):
    """The paper's entropy model for residuals (Sec. 3.3, inter-frame optimisation), used as a
    context-free baseline: per attribute a Gaussian with the symbols' mean and standard deviation,
    bits of the rint-quantised symbols under its PMF (CDF differences one step apart, floor 1e-9)."""
    from math import erf, sqrt
    out = np.zeros(attrs.shape[0])
    verf = np.vectorize(erf)
    for a in range(attrs.shape[0]):
        y = np.rint(attrs[a].astype(np.float64) / step) * step
        mu, sd = y.mean(), max(y.std(), step / 16)
        ks, cnt = np.unique(y, return_counts=True)
        hi = 0.5 * (1 + verf((ks + step / 2 - mu) / (sd * sqrt(2))))
        lo = 0.5 * (1 + verf((ks - step / 2 - mu) / (sd * sqrt(2))))
        P = np.maximum(hi - lo, 1e-9)
        out[a] = -(cnt * np.log2(P)).sum()
    return out
