"""Pins of the FP64 D-SSIM oracle: the window against scipy's Gaussian filter, SSIM against
brute-force window sums, closed forms (identical images, constant images), symmetry, the L1
limit, and the gradient against central finite differences."""
import numpy as np
import pytest
from scipy import ndimage

import oracle
from oracle import ssim as S


def _img(rng, *shape):
    return rng.uniform(0.0, 1.0, shape)


def test_window_is_scipy_gaussian_filter_with_zero_padding():
    rng = np.random.default_rng(1)
    x = _img(rng, 3, 23, 31)
    ref = np.stack([ndimage.gaussian_filter(x[c], S.SIGMA, mode="constant", cval=0.0,
                                            truncate=(S.WIN // 2) / S.SIGMA) for c in range(3)])
    np.testing.assert_allclose(S.blur(x), ref, rtol=1e-12, atol=1e-14)


def test_ssim_map_equals_brute_force_window_sums():
    rng = np.random.default_rng(2)
    x, y = _img(rng, 9, 14), _img(rng, 9, 14)
    g = S.window_1d()
    w2 = np.outer(g, g)
    r = S.WIN // 2
    xp = np.pad(x, r)
    yp = np.pad(y, r)
    Smap = S.ssim_parts(x, y)[0]
    for (i, j) in [(0, 0), (4, 7), (8, 13), (2, 11)]:
        wx, wy = xp[i:i + S.WIN, j:j + S.WIN], yp[i:i + S.WIN, j:j + S.WIN]
        m1, m2 = (w2 * wx).sum(), (w2 * wy).sum()
        v1 = (w2 * wx * wx).sum() - m1 * m1
        v2 = (w2 * wy * wy).sum() - m2 * m2
        c12 = (w2 * wx * wy).sum() - m1 * m2
        ref = (2 * m1 * m2 + S.C1) * (2 * c12 + S.C2) / ((m1 * m1 + m2 * m2 + S.C1) * (v1 + v2 + S.C2))
        assert abs(Smap[i, j] - ref) < 1e-12


def test_identical_images_have_ssim_one_and_no_dssim_gradient():
    rng = np.random.default_rng(3)
    y = _img(rng, 1, 3, 12, 10)
    x = np.stack([y, y], axis=1)
    loss, g = S.color_loss(x, y, [1.0, 0.5], 1.0)
    assert abs(loss) < 1e-14
    assert np.abs(g).max() < 1e-12
    np.testing.assert_allclose(S.ssim_parts(x[0, 0], x[0, 0])[0], 1.0, atol=1e-14)


def test_constant_images_closed_form_and_symmetry():
    a, b = 0.3, 0.8
    x = np.full((21, 25), a)
    y = np.full((21, 25), b)
    Smap = S.ssim_parts(x, y)[0]
    interior = Smap[5:-5, 5:-5]
    np.testing.assert_allclose(interior, (2 * a * b + S.C1) / (a * a + b * b + S.C1), rtol=1e-12)
    rng = np.random.default_rng(4)
    u, v = _img(rng, 11, 13), _img(rng, 11, 13)
    np.testing.assert_allclose(S.ssim_parts(u, v)[0], S.ssim_parts(v, u)[0], rtol=1e-12)


def test_lambda_zero_is_the_l1_loss():
    rng = np.random.default_rng(5)
    img = _img(rng, 2, 3, 3, 9, 12)
    tgt = _img(rng, 2, 3, 9, 12)
    lw = [0.5, 0.25, 1.0]
    loss, g = S.color_loss(img, tgt, lw, 0.0)
    assert abs(loss - oracle.l1_loss(img, tgt, lw)) < 1e-12
    np.testing.assert_allclose(g, oracle.l1_grad(img, tgt, lw), rtol=0, atol=1e-15)


@pytest.mark.parametrize("lam", [1.0, 0.2])
def test_gradient_matches_central_differences(lam):
    rng = np.random.default_rng(6)
    img = _img(rng, 1, 2, 3, 13, 17)
    tgt = _img(rng, 1, 3, 13, 17)
    lw = [0.5, 1.0]
    _, g = S.color_loss(img, tgt, lw, lam)
    h = 1e-6
    for _ in range(40):
        idx = tuple(rng.integers(0, s) for s in img.shape)
        if lam < 1.0 and abs(img[idx] - tgt[(idx[0],) + idx[2:]]) < 1e-3:
            continue  # the L1 kink
        p, m = img.copy(), img.copy()
        p[idx] += h
        m[idx] -= h
        fd = (S.color_loss(p, tgt, lw, lam)[0] - S.color_loss(m, tgt, lw, lam)[0]) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * abs(fd) + 1e-9, (idx, fd, g[idx])
