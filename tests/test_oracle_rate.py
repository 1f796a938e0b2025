"""Pins of the rate oracle: the discretised-Laplace PMF (Sec. 3.3, PMF from CDF differences)
against its definition, normalisation and entropy; the histogram rate against exact counts;
BF16 rounding and GELU against torch; the counter-based noise generator against the
SplitMix64 reference output; the MLP backward against finite differences."""
import math

import numpy as np
import torch

from oracle import rate

Q = 1.0 / 64


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10 ** rng.uniform(-6, 6, 20000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38])])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(rate.bf16_round(x32.astype(np.float64)), ref)
    bits = rate.f64_to_bf16_bits(x32.astype(np.float64))
    np.testing.assert_array_equal(rate.bf16_bits_to_f64(bits), ref)


def test_splitmix64_reference_output_and_uniformity():
    # first output of the SplitMix64 reference generator seeded with 0
    z = rate.splitmix64(np.uint64(0x9E3779B97F4A7C15))
    assert int(z) == 0xE220A8397B1DCDAF
    u = rate.noise(3, 100000, Q, seed=1234, offset=7) / Q + 0.5
    assert u.min() >= 0 and u.max() < 1
    # KS distance to U[0, 1)
    s = np.sort(u[1])
    ks = np.max(np.abs(s - np.arange(1, s.size + 1) / s.size))
    assert ks < 0.01
    # different counters give different streams
    assert not np.array_equal(rate.noise(1, 100, Q, 1, 0), rate.noise(1, 100, Q, 1, 100))


def test_laplace_pmf_sums_to_one_and_matches_bits():
    m, b = 0.123, 0.07
    k = np.arange(-20000, 20001)
    P = rate.laplace_pmf(k, m, b, Q)
    assert abs(P.sum() - 1.0) < 1e-12
    y = k[::97] * Q
    bits, _, _ = rate.laplace_bits(y, m, b, Q)
    ref = -np.log2(np.maximum(rate.laplace_pmf(k[::97], m, b, Q), 1e-9))
    np.testing.assert_allclose(bits, ref, rtol=1e-9, atol=1e-9)


def test_laplace_bits_gradients_fd():
    rng = np.random.default_rng(1)
    y = rng.normal(0, 0.3, 400)
    m = rng.normal(0, 0.3, 400)
    b = rng.uniform(0.005, 0.5, 400)
    bits, dy, db = rate.laplace_bits(y, m, b, Q)
    h = 1e-7
    fy = (rate.laplace_bits(y + h, m, b, Q)[0] - rate.laplace_bits(y - h, m, b, Q)[0]) / (2 * h)
    fb = (rate.laplace_bits(y, m, b + h, Q)[0] - rate.laplace_bits(y, m, b - h, Q)[0]) / (2 * h)
    ok = np.abs(np.abs(y - m) - Q / 2) > 1e-5  # away from the |y - m| = q/2 seam
    ok &= bits < 29.8
    np.testing.assert_allclose(dy[ok], fy[ok], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(db[ok], fb[ok], rtol=1e-5, atol=1e-5)


def test_histogram_bits_exact_counts_and_rounding():
    # symbols 0 (x1), 1 (x2), 2 (x5) -> -(1 log2 1/8 + 2 log2 2/8 + 5 log2 5/8)
    y = np.array([0.0, 1, 1, 2, 2, 2, 2, 2]) * Q
    exp = -(1 * math.log2(1 / 8) + 2 * math.log2(2 / 8) + 5 * math.log2(5 / 8))
    assert abs(rate.hist_bits(y[None].astype(np.float32), Q)[0] - exp) < 1e-12
    # ties round to even: 0.5 -> 0, 1.5 -> 2, 2.5 -> 2
    y2 = np.array([0.5, 1.5, 2.5, 2.0]) * Q
    # symbols {0, 2, 2, 2}
    exp2 = -(1 * math.log2(1 / 4) + 3 * math.log2(3 / 4))
    assert abs(rate.hist_bits(y2[None].astype(np.float32), Q)[0] - exp2) < 1e-12


def test_histogram_rate_of_laplace_data_is_its_discrete_entropy():
    rng = np.random.default_rng(2)
    m, b, N = 0.0, 0.2, 2_000_000
    y = rng.laplace(m, b, N).astype(np.float32)
    k = np.arange(-4000, 4001)
    P = rate.laplace_pmf(k, m, b, Q)
    H = -(P[P > 0] * np.log2(P[P > 0])).sum()
    hb = rate.hist_bits(y[None], Q)[0] / N
    assert abs(hb - H) < 0.01 * H
    # the matching Laplace model's mean rate is the same entropy (cross-entropy with the truth)
    lb = rate.laplace_bits(np.rint(y.astype(np.float64) / Q) * Q, m, b, Q)[0].mean()
    assert abs(lb - H) < 0.005 * H
    assert lb >= hb - 1e-3  # Gibbs: a context-free model cannot beat the empirical entropy (up to sampling)


def test_gelu_matches_torch_tanh_form():
    x = np.linspace(-8, 8, 2001)
    ref = torch.nn.functional.gelu(torch.from_numpy(x), approximate="tanh").numpy()
    np.testing.assert_allclose(rate.gelu(x), ref, atol=1e-14)
    h = 1e-6
    np.testing.assert_allclose(rate.gelu_grad(x), (rate.gelu(x + h) - rate.gelu(x - h)) / (2 * h), atol=1e-8)


def _mlp_case(seed=3, n=300, A=2):
    rng = np.random.default_rng(seed)
    attrs = rng.normal(0, 0.3, (A, n)).astype(np.float32)
    means = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    ctx = rate.context(means, 1.0, rate.layer_of(n, [100, 300]))
    wbits, bf = rate.init_weights(A, seed, attrs)
    wf = rate.bf16_bits_to_f64(wbits)
    return attrs, ctx, wbits, bf, wf


def test_mlp_weight_gradients_fd():
    attrs, ctx, wbits, bf, wf = _mlp_case()
    base = rate.rate_model(attrs, ctx, wbits, bf, Q, mode=0, emulate_bf16=False, weights_f64=wf)
    rng = np.random.default_rng(4)
    h = 1e-6
    for a in range(2):
        for j in rng.choice(rate.W_PER_ATTR, 40, replace=False):
            wp, wm = wf.copy(), wf.copy()
            wp[a, j] += h
            wm[a, j] -= h
            lp = rate.rate_model(attrs, ctx, wbits, bf, Q, emulate_bf16=False, weights_f64=wp, want_grad=False)["loss"]
            lm = rate.rate_model(attrs, ctx, wbits, bf, Q, emulate_bf16=False, weights_f64=wm, want_grad=False)["loss"]
            fd = (lp - lm) / (2 * h)
            g = base["d_w"][a, j]
            assert abs(g - fd) <= 1e-4 * abs(fd) + 1e-4, (a, j, g, fd)
        for j in range(rate.B_PER_ATTR):
            bp, bm = bf.astype(np.float64).copy(), bf.astype(np.float64).copy()
            bp[a, j] += h
            bm[a, j] -= h
            lp = rate.rate_model(attrs, ctx, wbits, bp, Q, emulate_bf16=False, weights_f64=wf, want_grad=False)["loss"]
            lm = rate.rate_model(attrs, ctx, wbits, bm, Q, emulate_bf16=False, weights_f64=wf, want_grad=False)["loss"]
            fd = (lp - lm) / (2 * h)
            assert abs(base["d_b"][a, j] - fd) <= 1e-4 * abs(fd) + 1e-4, (a, j)


def test_train_mode_attr_gradient_fd():
    attrs, ctx, wbits, bf, wf = _mlp_case(seed=5, n=200, A=1)
    w = rate.symbol_weights(200, [100, 200], [0.5, 1.0], 1e-2)
    base = rate.rate_model(attrs, ctx, wbits, bf, Q, mode=1, seed=9, offset=3, sym_w=w)
    h = 1e-4
    for i in range(0, 200, 17):
        ap, am = attrs.copy(), attrs.copy()
        ap[0, i] += h
        am[0, i] -= h
        dx = float(ap[0, i]) - float(am[0, i])
        lp = rate.rate_model(ap, ctx, wbits, bf, Q, mode=1, seed=9, offset=3, sym_w=w, want_grad=False)["loss"]
        lm = rate.rate_model(am, ctx, wbits, bf, Q, mode=1, seed=9, offset=3, sym_w=w, want_grad=False)["loss"]
        fd = (lp - lm) / dx
        assert abs(base["d_attrs"][0, i] - fd) <= 1e-3 * abs(fd) + 1e-9, (i, base["d_attrs"][0, i], fd)


def test_symbol_weights_and_layers():
    lo = rate.layer_of(10, [2, 5, 10])
    np.testing.assert_array_equal(lo, [1, 1, 2, 2, 2, 3, 3, 3, 3, 3])
    w = rate.symbol_weights(10, [2, 5, 10], [0.5, 0.25, 1.0], 2.0)
    np.testing.assert_allclose(w[:2], 0.5), np.testing.assert_allclose(w[2:5], 2 * 0.25 / 3)
    np.testing.assert_allclose(w[5:], 2 * 1.0 / 5)


def test_context_features_by_hand():
    """The 16 context features of the learned rate model (a reading: the MLP inputs are not given
    by the paper) at points whose sines and cosines are known exactly: u = mean / extent, then
    sin(pi u), cos(pi u), sin(2 pi u), cos(2 pi u) per axis, then (layer - 1) / 5, each rounded to
    BF16 (sqrt(2)/2 -> 0.70703125, 0.4 -> 0.400390625, 0.2 -> 0.2001953125)."""
    r = 0.70703125
    means = np.array([[0.5, 1.0], [-0.25, 0.0], [1.0, -0.5]])  # two Gaussians, columns
    layer = np.array([3, 2])
    got = rate.context(means, 1.0, layer)
    exp0 = [0.5, -0.25, 1.0,  1.0, -r, 0.0,  0.0, r, -1.0,  0.0, -1.0, 0.0,  -1.0, 0.0, 1.0,  0.400390625]
    exp1 = [1.0, 0.0, -0.5,  0.0, 0.0, -1.0,  -1.0, 1.0, 0.0,  0.0, 0.0, 0.0,  1.0, 1.0, -1.0,  0.2001953125]
    np.testing.assert_allclose(got[:, 0], exp0, atol=1e-15)
    np.testing.assert_allclose(got[:, 1], exp1, atol=1e-15)
    # the extent scales the positions: extent 2 halves u
    g2 = rate.context(2.0 * means, 2.0, layer)
    np.testing.assert_array_equal(g2, got)
    # layers from the nested level counts: Gaussian i belongs to the first level whose count exceeds i
    np.testing.assert_array_equal(rate.layer_of(10, [2, 5, 10]), [1, 1, 2, 2, 2, 3, 3, 3, 3, 3])


def test_context_free_fits_match_the_histogram_on_their_own_distributions():
    """The two context-free baselines of the gain test reach the empirical entropy (histogram bits)
    on data drawn from their own family and lose to it on the other family (Gibbs' inequality: the
    histogram is the least rate any context-free model can assign)."""
    rng = np.random.default_rng(0)
    y = np.stack([rng.laplace(0.1, 0.05, 200_000), rng.normal(-0.2, 0.07, 200_000)]).astype(np.float32)
    h = rate.hist_bits(y, 1 / 64)
    lap = rate.laplace_fit_bits(y, 1 / 64)
    gau = rate.gaussian_fit_bits(y, 1 / 64)
    assert abs(lap[0] / h[0] - 1) < 5e-3 and abs(gau[1] / h[1] - 1) < 5e-3
    assert lap[1] > 1.01 * h[1] and gau[0] > 1.01 * h[0]
    assert np.all(lap >= h) and np.all(gau >= h)


def test_bucketed_histogram_by_hand_and_its_bounds():
    """The bucketed histogram rate: a hand count on a tiny case, one bucket == the plain histogram,
    conditioning never adds bits, and buckets that split the symbols exactly remove them."""
    q = 1.0 / 64
    y = np.array([[0, 0, 1, 1, 1, 2]], np.float32) * q
    b = np.array([0, 0, 0, 1, 1, 1])
    # bucket 0 holds symbols {0: 2, 1: 1} of 3, bucket 1 {1: 2, 2: 1} of 3
    want = -(2 * math.log2(2 / 3) + math.log2(1 / 3)) * 2
    assert abs(rate.bucketed_hist_bits(y, q, b)[0] - want) < 1e-12
    rng = np.random.default_rng(4)
    a = rng.laplace(0, 0.1, (3, 5000)).astype(np.float32)
    one = rate.bucketed_hist_bits(a, q, np.zeros(5000, int))
    assert np.allclose(one, rate.hist_bits(a, q), rtol=0, atol=1e-6)
    bk = rng.integers(0, 16, 5000)
    assert np.all(rate.bucketed_hist_bits(a, q, bk) <= rate.hist_bits(a, q) + 1e-9)
    # a bucket equal to the symbol itself leaves nothing to code
    k = np.rint(a[0].astype(np.float64) / q).astype(np.int64)
    assert abs(rate.bucketed_hist_bits(a[:1], q, k)[0]) < 1e-9
    m = np.array([[-1.0, 1.0, -1.0, 1.0], [-1.0, -1.0, 1.0, 1.0], [1.0, 1.0, 1.0, -1.0]])
    assert list(rate.layer_octant_bucket(m, [1, 1, 2, 2])) == [8 + 4, 8 + 5, 16 + 6, 16 + 3]
