"""Pins of the entropy-model oracle (KDE of keyframe attributes, Gaussian of residuals): the
bandwidth against scipy's gaussian_kde with Silverman's rule, the binned grid CDF against scipy's
exact KDE CDF within the linear-binning error bound, the PMF telescoping to the CDF mass, the
Gaussian model against scipy's normal CDF, and both gradients against central differences."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import entropy as E

Q = 1.0 / 64


def _sym(n, seed, scale=0.3, mix=True):
    rng = np.random.default_rng(seed)
    y = rng.normal(0.0, scale, n)
    if mix:  # an irregular, two-mode density like the keyframe attributes
        y[: n // 3] = rng.normal(1.0, 0.05, n // 3)
    return np.rint(y / Q) * Q + rng.uniform(-Q / 2, Q / 2, n)


def test_bandwidth_is_scipy_silverman():
    y = _sym(3000, 1)
    kde = stats.gaussian_kde(y, bw_method="silverman")
    assert abs(E.silverman(y, Q) - kde.factor * np.std(y, ddof=1)) < 1e-12
    assert E.silverman(np.full(10, 0.25), Q) == Q / 4  # equal symbols: the floor


@pytest.mark.parametrize("seed,scale", [(2, 0.3), (3, 0.02)])
def test_grid_cdf_matches_exact_kde_within_binning_bound(seed, scale):
    y = _sym(2000, seed, scale)
    F, (h, lo, delta, G, K) = E.kde_cdf(y, Q)
    kde = stats.gaussian_kde(y, bw_method="silverman")
    assert abs(kde.factor * np.std(y, ddof=1) - h) < 1e-12 or h == Q / 4
    ks = np.linspace(0, G - 1, 60).astype(int)
    exact = np.array([np.mean(stats.norm.cdf((lo + k * delta - y) / h)) for k in ks])
    # linear binning moves each symbol's kernel by at most Delta: its CDF error is at most
    # Delta^2 / 8 times the largest second derivative of Phi(./h), phi'(1) / h^2
    bound = delta ** 2 / 8 * 0.2420 / h ** 2
    assert np.abs(F[ks] - exact).max() <= bound + 1e-12
    # and the exact KDE CDF from scipy at a few points
    for x in (-0.4, 0.0, 0.3, 1.0):
        val, _ = E._interp(F, lo, delta, np.array([x]))
        ref = kde.integrate_box_1d(-np.inf, x)
        assert abs(val[0] - ref) <= bound + delta ** 2 / (8 * h ** 2 * math.sqrt(2 * math.pi)) + 1e-9


def test_pmf_telescopes_and_is_a_probability():
    y = _sym(1500, 4)
    F, (h, lo, delta, G, K) = E.kde_cdf(y, Q)
    assert F[0] < 1e-12 and abs(F[-1] - 1.0) < 1e-9 and np.all(np.diff(F) >= -1e-15)
    centres = lo + 2 * Q + Q * np.arange(int((G - 1) * delta / Q) - 4)
    Fp, _ = E._interp(F, lo, delta, centres + Q / 2)
    Fm, _ = E._interp(F, lo, delta, centres - Q / 2)
    P = Fp - Fm
    assert np.all(P >= -1e-15) and abs(P.sum() - 1.0) < 1e-9


def test_kde_gradient_with_the_density_held_fixed():
    y = _sym(800, 5)
    F, (h, lo, delta, G, K) = E.kde_cdf(y, Q)
    bits, db = E.kde_bits(y, Q)

    def b_at(x):
        Fp, _ = E._interp(F, lo, delta, x + Q / 2)
        Fm, _ = E._interp(F, lo, delta, x - Q / 2)
        return -np.log2(np.maximum(Fp - Fm, E.P_FLOOR))

    assert np.allclose(b_at(y), bits, rtol=0, atol=1e-12)
    eps = 1e-3 * delta  # inside one grid segment (where the CDF is linear) for most symbols
    fd = (b_at(y + eps) - b_at(y - eps)) / (2 * eps)
    t = ((y - lo) / delta) % 1.0
    tp = ((y + Q / 2 - lo) / delta) % 1.0
    tm = ((y - Q / 2 - lo) / delta) % 1.0
    ok = np.minimum.reduce([np.minimum(t, 1 - t), np.minimum(tp, 1 - tp), np.minimum(tm, 1 - tm)]) > 2e-3
    assert ok.sum() > 700
    assert np.allclose(fd[ok], db[ok], rtol=1e-5, atol=1e-6)


def test_gaussian_model_closed_form_and_total_gradient():
    rng = np.random.default_rng(6)
    y = rng.normal(0.01, 0.02, 700)
    bits, total, direct = E.gaussian_bits(y, Q)
    mu, sd = y.mean(), y.std()
    ref = -np.log2(stats.norm.cdf(y + Q / 2, mu, sd) - stats.norm.cdf(y - Q / 2, mu, sd))
    assert np.allclose(bits, ref, rtol=1e-10, atol=1e-10)
    # the gradient of sum_i bits_i, mu and sigma moving with every symbol
    for k in (0, 17, 350, 699):
        e = 1e-6
        yp, ym = y.copy(), y.copy()
        yp[k] += e
        ym[k] -= e
        fd = (E.gaussian_bits(yp, Q)[0].sum() - E.gaussian_bits(ym, Q)[0].sum()) / (2 * e)
        assert abs(fd - total[k]) <= 1e-5 * abs(fd) + 1e-6, (k, fd, total[k])
        assert abs(direct[k] - total[k]) > 1e-3 * abs(total[k])  # the mu / sigma terms matter


def test_tail_symbols_hit_the_floor_with_zero_gradient():
    y = np.concatenate([np.zeros(999), [40.0]])
    bits, total, direct = E.gaussian_bits(y, Q)
    assert abs(bits[-1] + math.log2(E.P_FLOOR)) < 1e-9 and direct[-1] == 0.0


def test_entropy_model_symbols_loss_and_layers():
    rng = np.random.default_rng(7)
    attrs = rng.normal(0, 0.2, (3, 900)).astype(np.float32)
    sym = E.symbols(attrs, Q, 0)
    assert np.allclose(sym, np.rint(attrs.astype(np.float64) / np.float32(Q)) * np.float32(Q), atol=1e-9)
    lv, lw = [300, 900], [0.5, 1.0]
    bits, loss, per, grad = E.entropy_model(attrs, Q, 1, mode=1, seed=3, offset=5, level_counts=lv,
                                            level_weights=lw, lambda_rate=2.0, lambda_reg=0.1)
    y = E.symbols(attrs, Q, 1, 3, 5)
    exp = 2.0 * (0.5 * per[:, :300].sum() / 300 + per[:, 300:].sum() / 600) + \
        0.1 * (0.5 * np.abs(y[:, :300]).sum() + np.abs(y[:, 300:]).sum())
    assert abs(loss - exp) < 1e-9 * exp
    assert np.allclose(bits, per.sum(axis=1))
    # each layer's density is its own: changing layer 1 leaves layer 0's bits alone
    attrs2 = attrs.copy()
    attrs2[:, 400:] += 0.5
    _, _, per2, _ = E.entropy_model(attrs2, Q, 0, level_counts=lv)
    _, _, per0, _ = E.entropy_model(attrs, Q, 0, level_counts=lv)
    assert np.array_equal(per2[:, :300], per0[:, :300]) and not np.allclose(per2[:, 300:], per0[:, 300:])
