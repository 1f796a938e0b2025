"""Pins of the oracle's analytic backward: FP64 central finite differences of
L = sum(w * image) on tiny scenes (every parameter, including frame residuals
and several levels), and single-Gaussian closed forms. A parameter whose
perturbation changes a discrete event of the forward (the included set, the
stop position, an alpha / colour / Jacobian clamp) is re-tried at a smaller
step and otherwise skipped and counted.

Paper passages: differentiable splatting of Eq. 2 / Eq. 4 (Sec. 3.1) and the
frame composition of Sec. 3.2.
"""
import math

import numpy as np
import pytest

import oracle
import synth

Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def _loss(st, p, cams, F, res, w):
    r = oracle.render(st, p, cams, n_frames=F, residuals=res, signature=True)
    flags = oracle.project(st, p, cams, F, res)[:, :, [0, 15]]
    return float((r["image"] * w).sum()), r["sig"], flags


def _fd_check(st, p, cams, w, F=1, res=None, h=1e-4, sample=None, target="params"):
    """Returns (n_checked, n_skipped, worst relative error)."""
    dp, dr, _ = oracle.backward(st, p, cams, w, n_frames=F, residuals=res)
    arr = p if target == "params" else res
    grad = dp if target == "params" else dr
    idxs = list(np.ndindex(arr.shape)) if sample is None else sample
    checked = skipped = 0
    worst = 0.0
    scale = np.sqrt(np.mean(grad ** 2)) + 1e-30
    for ix in idxs:
        ok = False
        for hh in (h, h / 10):
            ap, am = arr.copy(), arr.copy()
            ap[ix] = np.float32(arr[ix] + hh)
            am[ix] = np.float32(arr[ix] - hh)
            dx = float(ap[ix]) - float(am[ix])
            if target == "params":
                lp, sp, fp = _loss(st, ap, cams, F, res, w)
                lm, sm, fm = _loss(st, am, cams, F, res, w)
            else:
                lp, sp, fp = _loss(st, p, cams, F, ap, w)
                lm, sm, fm = _loss(st, p, cams, F, am, w)
            if np.array_equal(sp, sm) and np.array_equal(fp, fm):
                ok = True
                break
        if not ok:
            skipped += 1
            continue
        fd = (lp - lm) / dx
        g = grad[ix]
        err = abs(g - fd) / (abs(fd) + 1e-3 * scale)
        worst = max(worst, err)
        checked += 1
    return checked, skipped, worst


def _tiny(seed, n=12, deg=3, wdt=24, hgt=20, n_views=2):
    p = synth.cube_scene(n, seed, deg)
    p[3:6] += 1.2  # larger footprints so that every Gaussian covers pixels of the small image
    cams = synth.ring_cameras(list(range(0, 24, 24 // n_views))[:n_views], 24, 4.0, wdt, hgt, float(wdt))
    return p, cams


def test_fd_all_params_sh3_two_views_three_levels():
    p, cams = _tiny(21)
    st = oracle.Settings(24, 20, 3, (4, 8, 12), dilation=0.3)
    w = np.random.default_rng(22).standard_normal((2, 3, 3, 20, 24))
    checked, skipped, worst = _fd_check(st, p, cams, w)
    assert checked >= 0.9 * p.size, (checked, skipped)
    assert worst < 1e-5, worst


def test_fd_background_and_clamped_alpha():
    p, cams = _tiny(23, n=10, deg=1)
    p[10, :3] = 8.0  # o ~ 0.9997: alpha clamped at the centre
    st = oracle.Settings(24, 20, 1, (10,), dilation=0.3, bg=(0.2, 0.5, 0.9))
    w = np.random.default_rng(24).standard_normal((2, 1, 3, 20, 24))
    checked, skipped, worst = _fd_check(st, p, cams, w)
    assert checked >= 0.85 * p.size, (checked, skipped)
    assert worst < 1e-5, worst


def test_fd_frame_residuals():
    n, F = 8, 3
    p, cams1 = _tiny(25, n=n, deg=1)
    C = p.shape[0]
    res = synth.frame_residuals(n, F, 26, channels=C, sd_mean=0.05, sd_angle=0.3, sd_logit=0.3,
                                sd_log_scale=0.1, sd_sh=0.1)
    cams = np.concatenate([cams1] * F)
    st = oracle.Settings(24, 20, 1, (n,), dilation=0.3, res_channels=C)
    w = np.random.default_rng(27).standard_normal((F * 2, 1, 3, 20, 24))
    c1, s1, w1 = _fd_check(st, p, cams, w, F=F, res=res)
    assert c1 >= 0.85 * p.size and w1 < 1e-5, (c1, s1, w1)
    c2, s2, w2 = _fd_check(st, p, cams, w, F=F, res=res, target="res")
    assert c2 >= 0.85 * res.size and w2 < 1e-5, (c2, s2, w2)


def test_fd_rigid_residuals_only():
    n, F = 8, 2
    p, cams1 = _tiny(28, n=n, deg=0)
    res = synth.frame_residuals(n, F, 29, channels=8, sd_mean=0.05, sd_angle=0.3, sd_logit=0.3)
    cams = np.concatenate([cams1] * F)
    st = oracle.Settings(24, 20, 0, (n,), dilation=0.3, res_channels=8)
    w = np.random.default_rng(30).standard_normal((F * 2, 1, 3, 20, 24))
    c2, s2, w2 = _fd_check(st, p, cams, w, F=F, res=res, target="res")
    assert c2 >= 0.85 * res.size and w2 < 1e-5, (c2, s2, w2)


def test_single_gaussian_closed_form_gradients():
    """dC/dlogit = c G sigma (1 - sigma) (unclamped alpha) and dC/df_dc = alpha Y00."""
    z, sig, o = 3.0, 0.1, 0.6
    p = np.zeros((14, 1), np.float32)
    p[0:3, 0] = [0.0, 0.0, z]
    p[3:6, 0] = math.log(sig)
    p[6, 0] = 1.0
    p[10, 0] = math.log(o / (1 - o))
    p[11:14, 0] = [0.4, 0.1, -0.3]
    Wd = Hd = 16
    cams = synth.identity_camera(Wd, Hd, 16.0)[None]
    st = oracle.Settings(Wd, Hd, 0, (1,), dilation=0.3)
    pr = oracle.project(st, p, cams)[0, 0]
    px, py = 9, 6
    w = np.zeros((1, 1, 3, Hd, Wd))
    w[0, 0, 0, py, px] = 1.0  # red channel of one pixel
    dp, _, _ = oracle.backward(st, p, cams, w)
    dx, dy = px + 0.5 - pr[2], py + 0.5 - pr[3]
    G = math.exp(-0.5 * (pr[7] * dx * dx + 2 * pr[8] * dx * dy + pr[9] * dy * dy))
    s = pr[10]
    np.testing.assert_allclose(dp[10, 0], pr[11] * G * s * (1 - s), rtol=1e-12)
    np.testing.assert_allclose(dp[11, 0], s * G * Y00, rtol=1e-12)
    assert dp[12, 0] == 0.0 and dp[13, 0] == 0.0


def test_footprint_local_fd_equals_analytic_and_full_render_fd():
    """O8's footprint-local differences (only the pixels the perturbed Gaussian can reach are
    re-composited, kinks handled per pixel-level) agree with the analytic backward on every
    parameter of a tiny scene, and with differences of full re-renders where those are smooth."""
    p, cams = _tiny(31, n=14, deg=3)
    st = oracle.Settings(24, 20, 3, (5, 14), dilation=0.3)
    w = np.random.default_rng(32).standard_normal((2, 2, 3, 20, 24))
    dp, _, _ = oracle.backward(st, p, cams, w)
    C, n = p.shape
    gi, ci = np.meshgrid(np.arange(n), np.arange(C))
    fd, status, skipped = oracle.finite_differences(st, p, cams, w, gi.ravel(), ci.ravel(), h=1e-5)
    fd = fd.reshape(C, n)
    assert np.all(status & 8 == 0)
    ok = (status.reshape(C, n) & 4) == 0
    assert ok.mean() > 0.95
    scale = np.sqrt(np.mean(dp ** 2))
    err = np.abs(fd - dp) / (np.abs(dp) + 1e-3 * scale)
    assert err[ok].max() < 1e-5, err[ok].max()
    # full-render differences of a few smooth parameters (float32 steps, so the step is the
    # float32 difference of the perturbed values)
    for ch, i in ((0, 3), (4, 5), (7, 8), (10, 2), (20, 9)):
        ap, am = p.copy(), p.copy()
        ap[ch, i] = np.float32(p[ch, i] + 1e-3)
        am[ch, i] = np.float32(p[ch, i] - 1e-3)
        lp = float((oracle.render(st, ap, cams)["image"] * w).sum())
        lm = float((oracle.render(st, am, cams)["image"] * w).sum())
        full = (lp - lm) / (float(ap[ch, i]) - float(am[ch, i]))
        assert abs(full - fd[ch, i]) <= 1e-3 * abs(fd[ch, i]) + 1e-4 * scale, (ch, i, full, fd[ch, i])


def test_footprint_local_fd_kinks_fall_back_to_one_sided_differences():
    """A Gaussian whose alpha crosses alpha_min at some pixel between theta - h and theta + h:
    that pixel-level uses the side that keeps its events, so the difference still matches the
    analytic gradient (which differentiates the smooth part)."""
    p, cams = _tiny(33, n=10, deg=0)
    st = oracle.Settings(24, 20, 0, (10,), dilation=0.3)
    w = np.random.default_rng(34).standard_normal((2, 1, 3, 20, 24))
    dp, _, _ = oracle.backward(st, p, cams, w)
    C, n = p.shape
    gi, ci = np.meshgrid(np.arange(n), np.arange(C))
    fd, status, _ = oracle.finite_differences(st, p, cams, w, gi.ravel(), ci.ravel(), h=3e-2)
    fd, status = fd.reshape(C, n), status.reshape(C, n)
    one_sided = (status & 1) != 0
    assert one_sided.any()  # a large step makes kinks common
    ok = (status & 4) == 0
    scale = np.sqrt(np.mean(dp ** 2))
    # one-sided differences at a large step carry an O(h) error: compare loosely
    err = np.abs(fd - dp) / (np.abs(dp) + 1e-2 * scale)
    assert np.median(err[ok]) < 2e-2


def test_absolute_term_sums_bound_the_gradient_and_match_its_value():
    """backward_abs returns the analytic gradient unchanged and, beside it, the same sums taken of
    the absolute values of their terms, which bound it (|sum| <= sum |terms|) and equal it where
    no term can be negative (a one-pixel red weight on a single Gaussian's colour: dC/df_dc)."""
    p, cams = _tiny(41, n=9, deg=1)
    st = oracle.Settings(24, 20, 1, (9,), dilation=0.3)
    w = np.random.default_rng(42).standard_normal((2, 1, 3, 20, 24))
    dp, da = oracle.backward_abs(st, p, cams, w)
    dp2, _, _ = oracle.backward(st, p, cams, w)
    np.testing.assert_allclose(dp, dp2, rtol=1e-12, atol=1e-15)  # thread partial sums may add in another order
    assert np.all(da >= np.abs(dp) * (1 - 1e-12))
    w1 = np.zeros_like(w)
    w1[0, 0, 0] = 1.0  # red channel of view 0, every pixel, positive
    dp1, da1 = oracle.backward_abs(st, p, cams, w1)
    np.testing.assert_allclose(da1[11], np.abs(dp1[11]), rtol=1e-12)  # dC_r / df_dc,r = alpha T Y00 >= 0
