"""Pins of the FP64 oracle against facts it does not compute itself: closed forms of
the projection and of the compositing rule, library routines (scipy's complex
spherical harmonics and rotations), invariances, brute force and finite differences.

Paper passages: Gaussian density and covariance factorisation (Sec. 3.1, Eq. 1),
front-to-back compositing (Eq. 2), progressive rendering of nested layers
(Eq. 4), frame composition (Sec. 3.2, pose update and Eq. 7).
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.special import sph_harm_y

import oracle
import synth

Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def scene(means, log_scales, quats, logits, rgb, deg=0, extra_sh=None):
    """Explicit Gaussians -> params [C][N] (degree-0 colour rgb, i.e. f_dc = (rgb-0.5)/Y00)."""
    n = len(means)
    C = 11 + 3 * (deg + 1) ** 2
    p = np.zeros((C, n), np.float32)
    p[0:3] = np.asarray(means, np.float64).T
    p[3:6] = np.asarray(log_scales, np.float64).T
    p[6:10] = np.asarray(quats, np.float64).T
    p[10] = logits
    p[11:14] = ((np.asarray(rgb, np.float64) - 0.5) / Y00).T
    if extra_sh is not None:
        p[14:] = extra_sh
    return p


def logit(o):
    return math.log(o / (1.0 - o))


def f32(x):
    return float(np.float32(x))


W = H = 64
FOC = 64.0


def cam0(w=W, h=H, f=FOC):
    return synth.identity_camera(w, h, f)[None]


# ----------------------------------------------------------------- projection
@pytest.mark.parametrize("dil", [0.0, 0.3])
def test_isotropic_footprint_closed_form(dil):
    """Single isotropic Gaussian on the optical axis: Sigma2D = ((f sigma / z)^2 + d) I, so the
    image is c * min(0.99, o exp(-r^2 / (2 var))) where that is >= 1/255, else 0."""
    sig, z, o, c = 0.05, 3.0, 0.8, (0.7, 0.3, 0.9)
    p = scene([[0, 0, z]], [[math.log(sig)] * 3], [[1, 0, 0, 0]], [logit(o)], [c])
    st = oracle.Settings(W, H, 0, (1,), dilation=dil)
    img = oracle.render(st, p, cam0())["image"][0, 0]
    # exact values of the float32 inputs
    sig32, z32, o32 = math.exp(f32(math.log(sig))), f32(z), 1 / (1 + math.exp(-f32(logit(o))))
    c32 = [f32((ci - 0.5) / Y00) * Y00 + 0.5 for ci in c]
    var = (FOC * sig32 / z32) ** 2 + f32(dil)
    u = np.arange(W) + 0.5 - W / 2
    v = np.arange(H) + 0.5 - H / 2
    r2 = v[:, None] ** 2 + u[None, :] ** 2
    a = np.minimum(f32(0.99), o32 * np.exp(-r2 / (2 * var)))
    a[a < f32(1 / 255)] = 0.0
    for ch in range(3):
        np.testing.assert_allclose(img[ch], c32[ch] * a, rtol=0, atol=1e-12)


def test_offaxis_covariance_closed_form():
    """Isotropic Gaussian at camera-space (tx, 0, tz), unclamped Jacobian:
    Sigma2D = diag(f^2 s^2 (tz^2 + tx^2) / tz^4 + d, f^2 s^2 / tz^2 + d)."""
    s, tx, tz = 0.1, 0.8, 4.0
    p = scene([[tx, 0, tz]], [[math.log(s)] * 3], [[1, 0, 0, 0]], [0.0], [[0.5] * 3])
    st = oracle.Settings(W, H, 0, (1,), dilation=0.3)
    pr = oracle.project(st, p, cam0())[0, 0]
    s, tx, tz, d = math.exp(f32(math.log(s))), f32(tx), f32(tz), f32(0.3)
    assert pr[0] == 1.0
    np.testing.assert_allclose(pr[4], FOC ** 2 * s ** 2 * (tz ** 2 + tx ** 2) / tz ** 4 + d, rtol=1e-12)
    np.testing.assert_allclose(pr[5], 0.0, atol=1e-12)
    np.testing.assert_allclose(pr[6], FOC ** 2 * s ** 2 / tz ** 2 + d, rtol=1e-12)
    np.testing.assert_allclose(pr[2], FOC * tx / tz + W / 2, rtol=1e-12)
    # conic is the inverse of the covariance
    cov = np.array([[pr[4], pr[5]], [pr[5], pr[6]]])
    con = np.array([[pr[7], pr[8]], [pr[8], pr[9]]])
    np.testing.assert_allclose(con @ cov, np.eye(2), atol=1e-12)


@pytest.mark.parametrize("angle_deg", [0.0, 90.0, 30.0])
def test_anisotropic_axis_and_rotation(angle_deg):
    """Axis-aligned scales (a, b, c) on the axis rotated by theta about the optical axis:
    Sigma2D = (f/z)^2 Rot(theta) diag(a^2, b^2) Rot(theta)^T + d I."""
    a, b, c, z = 0.12, 0.04, 0.07, 3.0
    th = math.radians(angle_deg)
    q = [math.cos(th / 2), 0, 0, math.sin(th / 2)]
    p = scene([[0, 0, z]], [[math.log(a), math.log(b), math.log(c)]], [q], [0.0], [[0.5] * 3])
    st = oracle.Settings(W, H, 0, (1,), dilation=0.3)
    pr = oracle.project(st, p, cam0())[0, 0]
    a32, b32, z32 = math.exp(f32(math.log(a))), math.exp(f32(math.log(b))), f32(z)
    qq = np.array([f32(v) for v in q], np.float64)
    qq /= np.linalg.norm(qq)
    th32 = 2 * math.atan2(qq[3], qq[0])
    Rm = np.array([[math.cos(th32), -math.sin(th32)], [math.sin(th32), math.cos(th32)]])
    exp_cov = (FOC / z32) ** 2 * Rm @ np.diag([a32 ** 2, b32 ** 2]) @ Rm.T + f32(0.3) * np.eye(2)
    np.testing.assert_allclose([pr[4], pr[5], pr[6]], [exp_cov[0, 0], exp_cov[0, 1], exp_cov[1, 1]],
                               rtol=1e-12, atol=1e-12)


def test_quaternion_rotation_matches_scipy():
    rng = np.random.default_rng(0)
    for _ in range(20):
        q = rng.standard_normal(4)
        R = oracle.quat_rot(q)
        ref = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()  # scipy is scalar-last
        np.testing.assert_allclose(R, ref, atol=1e-13)


def test_quaternion_product_matches_rotation_composition():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a, b = rng.standard_normal(4), rng.standard_normal(4)
        ab = oracle.quat_mul(a, b)
        np.testing.assert_allclose(oracle.quat_rot(ab), oracle.quat_rot(a) @ oracle.quat_rot(b), atol=1e-12)
        sa = Rotation.from_quat([a[1], a[2], a[3], a[0]])
        sb = Rotation.from_quat([b[1], b[2], b[3], b[0]])
        np.testing.assert_allclose(oracle.quat_rot(ab), (sa * sb).as_matrix(), atol=1e-12)


# ------------------------------------------------------------- SH basis
def _real_sh_scipy(l, m, d):
    """Real SH with the Condon-Shortley phase kept: sqrt(2) Re / Im of the complex one."""
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    if m == 0:
        return sph_harm_y(l, 0, theta, phi).real
    if m > 0:
        return math.sqrt(2) * sph_harm_y(l, m, theta, phi).real
    return math.sqrt(2) * sph_harm_y(l, -m, theta, phi).imag


def test_sh_basis_matches_scipy_complex_harmonics():
    rng = np.random.default_rng(2)
    for _ in range(50):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        Y = oracle.sh_basis(3, d)
        for l in range(4):
            for m in range(-l, l + 1):
                np.testing.assert_allclose(Y[l * l + l + m], _real_sh_scipy(l, m, d), atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    nt, nph = 48, 96
    xg, wg = np.polynomial.legendre.leggauss(nt)  # cos(theta) nodes
    G = np.zeros((16, 16))
    for ct, wt in zip(xg, wg):
        st_ = math.sqrt(1 - ct * ct)
        for k in range(nph):
            ph = 2 * math.pi * k / nph
            Y = oracle.sh_basis(3, (st_ * math.cos(ph), st_ * math.sin(ph), ct))
            G += np.outer(Y, Y) * wt * (2 * math.pi / nph)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-6)


def test_degree0_view_independent_and_dc_gradient():
    p = scene([[0.2, -0.1, 3.0]], [[-2.0] * 3], [[1, 0, 0, 0]], [0.5], [[0.3, 0.6, 0.9]])
    cams = synth.ring_cameras([0, 5, 11], 24, 4.0, W, H, FOC)
    st = oracle.Settings(W, H, 0, (1,))
    pr = oracle.project(st, p, cams)
    assert np.all(pr[:, 0, 0] == 1.0)
    np.testing.assert_allclose(pr[:, 0, 11:14], np.broadcast_to(pr[0, 0, 11:14], (3, 3)), atol=1e-15)


# ------------------------------------------------------------ compositing
def _big(z, o, rgb):
    """A Gaussian much larger than the image (G ~ 1 at every pixel)."""
    return [0, 0, z], [math.log(1e4)] * 3, [1, 0, 0, 0], logit(o), rgb


def _stack(items, deg=0):
    m, s, q, lg, c = zip(*items)
    return scene(m, s, q, lg, c, deg)


def test_two_layers_closed_form():
    """C = c1 a1 + c2 a2 (1 - a1) (Eq. 2 with two Gaussians)."""
    sig = 0.08
    p = scene([[0, 0, 2.0], [0.05, 0, 3.0]], [[math.log(sig)] * 3, [math.log(0.12)] * 3],
              [[1, 0, 0, 0]] * 2, [logit(0.7), logit(0.6)], [[0.9, 0.2, 0.1], [0.1, 0.8, 0.4]])
    st = oracle.Settings(W, H, 0, (2,), dilation=0.3)
    img = oracle.render(st, p, cam0())["image"][0, 0]
    pr = oracle.project(st, p, cam0())[0]
    u = np.arange(W) + 0.5
    v = np.arange(H) + 0.5
    al = []
    for i in range(2):
        dx = u[None, :] - pr[i, 2]
        dy = v[:, None] - pr[i, 3]
        pw = -0.5 * (pr[i, 7] * dx * dx + 2 * pr[i, 8] * dx * dy + pr[i, 9] * dy * dy)
        a = np.minimum(f32(0.99), pr[i, 10] * np.exp(pw))
        a[a < f32(1 / 255)] = 0
        al.append(a)
    for ch in range(3):
        exp = pr[0, 11 + ch] * al[0] + pr[1, 11 + ch] * al[1] * (1 - al[0])
        np.testing.assert_allclose(img[ch], exp, atol=1e-12)


def test_full_occlusion():
    """a1 = 0.99 (clamped), a2 = 0.98: T = 2e-4 after two layers, so any layer behind with
    alpha > 0.5 stops the traversal and contributes exactly nothing (also zero gradient)."""
    items = [_big(2.0, 0.999, [0.8, 0.1, 0.3]), _big(3.0, 0.98, [0.2, 0.9, 0.5]),
             _big(4.0, 0.9, [0.4, 0.4, 0.9]), _big(5.0, 0.7, [1.0, 1.0, 1.0])]
    p = _stack(items)
    st = oracle.Settings(W, H, 0, (4,))
    r = oracle.render(st, p, cam0())
    img, T, nc = r["image"][0, 0], r["T"][0, 0], r["ncontrib"][0, 0]
    pr = oracle.project(st, p, cam0())[0]
    assert np.all(nc == 2)
    for ch in range(3):
        np.testing.assert_allclose(img[ch], 0.99 * pr[0, 11 + ch] + 0.0098 * pr[1, 11 + ch], atol=1e-7)
    np.testing.assert_allclose(T, 2e-4, rtol=1e-6)
    dimg = np.random.default_rng(3).standard_normal((1, 1, 3, H, W))
    dp, _, g2 = oracle.backward(st, p, cam0(), dimg)
    assert np.all(dp[:, 2:] == 0.0)
    assert np.all(g2[0, 2:] == 0.0)


def test_transmittance_stop_thirteen_layers():
    """k nested full-screen layers with alpha ~ 0.5: exactly 13 are included
    (2^-13 >= 1e-4 > 2^-14) and C = c (1 - 2^-13)."""
    c = [0.3, 0.6, 0.9]
    items = [_big(2.0 + 0.1 * k, 0.5, c) for k in range(20)]
    p = _stack(items)
    st = oracle.Settings(W, H, 0, (20,))
    r = oracle.render(st, p, cam0())
    assert np.all(r["ncontrib"][0, 0] == 13)
    pr = oracle.project(st, p, cam0())[0]
    a = pr[0, 10]
    for ch in range(3):
        np.testing.assert_allclose(r["image"][0, 0, ch], pr[0, 11 + ch] * (1 - 2.0 ** -13), atol=1e-8)
    assert abs(a - 0.5) < 1e-6


def test_alpha_cutoff_leaves_image_and_gradients():
    """A Gaussian with o < 1/255 never reaches the cutoff: the image is bit-identical without it
    and its gradient is exactly zero."""
    w = synth.config_plain_forward(seed=5, n=64, width=32, height=32)
    p = w.params.copy()
    p[10, 7] = logit(0.9 / 255)
    st = oracle.Settings(32, 32, 0, (64,))
    cams = synth.identity_camera(32, 32, 32.0)[None]
    img = oracle.render(st, p, cams)["image"]
    keep = np.ones(64, bool)
    keep[7] = False
    st2 = oracle.Settings(32, 32, 0, (63,))
    img2 = oracle.render(st2, p[:, keep], cams)["image"]
    assert np.array_equal(img, img2)
    dimg = np.random.default_rng(4).standard_normal(img.shape)
    dp, _, _ = oracle.backward(st, p, cams, dimg)
    assert np.all(dp[:, 7] == 0.0)


def test_brute_force_equals_bucketed():
    w = synth.config_plain_forward(seed=6, n=512, width=48, height=40)
    cams = synth.identity_camera(48, 40, 48.0)[None]
    st = oracle.Settings(48, 40, 0, (100, 300, 512))
    a = oracle.render(st, w.params, cams, mode="bucket")
    b = oracle.render(st, w.params, cams, mode="brute")
    for k in ("image", "T", "ncontrib"):
        assert np.array_equal(a[k], b[k])


def test_permutation_invariance():
    w = synth.config_plain_forward(seed=7, n=400, width=40, height=40)
    cams = synth.identity_camera(40, 40, 40.0)[None]
    st = oracle.Settings(40, 40, 0, (400,))
    a = oracle.render(st, w.params, cams)["image"]
    perm = np.random.default_rng(8).permutation(400)
    b = oracle.render(st, w.params[:, perm], cams)["image"]
    np.testing.assert_allclose(a, b, atol=1e-13)


def test_levels_equal_prefix_renders():
    """Eq. 4: level l composites only the first N_l Gaussians."""
    w = synth.config_plain_forward(seed=9, n=300, width=40, height=32)
    cams = synth.identity_camera(40, 32, 40.0)[None]
    lv = (25, 100, 300)
    r = oracle.render(oracle.Settings(40, 32, 0, lv), w.params, cams)["image"]
    for l, nl in enumerate(lv):
        rl = oracle.render(oracle.Settings(40, 32, 0, (nl,)), w.params[:, :nl], cams)["image"]
        assert np.array_equal(r[0, l], rl[0, 0])


def test_rigid_motion_invariance():
    """Moving every Gaussian and the camera by one rigid motion leaves a degree-0 image unchanged."""
    w = synth.config_plain_forward(seed=10, n=300, width=40, height=40)
    cams = synth.identity_camera(40, 40, 40.0)[None].astype(np.float64)
    st = oracle.Settings(40, 40, 0, (300,), dilation=0.3)
    a = oracle.render(st, w.params, cams)
    Q = Rotation.from_euler("xyz", [0.3, -0.2, 0.5])
    t = np.array([0.25, -0.5, 1.0])
    p = w.params.astype(np.float64).copy()
    p[0:3] = Q.apply(p[0:3].T).T + t[:, None]
    rq = (Q * Rotation.from_quat(np.stack([p[7], p[8], p[9], p[6]], 1))).as_quat()
    p[6:10] = np.stack([rq[:, 3], rq[:, 0], rq[:, 1], rq[:, 2]])
    Rm = Q.as_matrix()
    c = cams[0].copy()
    Rc = c[:12].reshape(3, 4)[:, :3]
    tc = c[:12].reshape(3, 4)[:, 3]
    Rn = Rc @ Rm.T
    tn = tc - Rn @ t
    c[:12] = np.concatenate([Rn, tn[:, None]], 1).reshape(-1)
    # the float32 depth key changes rounding; compare away from ambiguous pixels
    b = oracle.render(st, p.astype(np.float32), c[None].astype(np.float32), variants=True)
    ok = (b["nvar"] == 0) & (a["ncontrib"] == b["ncontrib"])
    assert ok.mean() > 0.97
    d = np.abs(a["image"] - b["image"]).max(axis=2)
    assert d[ok].max() < 2e-5


def test_frame_composition_equals_plain_render():
    """Frame f of a group = plain render of the keyframe composed with the deltas of frames 0..f
    (Sec. 3.2: mu_t = mu_{t-1} + d mu_t, R_t = dR_t R_{t-1}, Eq. 7 additive residuals)."""
    n, F = 200, 3
    p = synth.cube_scene(n, 11, 1)
    res = synth.frame_residuals(n, F, 12, channels=11 + 3 * 4, sd_mean=0.05, sd_angle=0.3,
                                sd_logit=0.3, sd_log_scale=0.1, sd_sh=0.1)
    cams1 = synth.ring_cameras([0, 7], 24, 4.0, 48, 32, 48.0)
    cams = np.concatenate([cams1] * F)
    st = oracle.Settings(48, 32, 1, (n,), res_channels=res.shape[1])
    r = oracle.render(st, p, cams, n_frames=F, residuals=res)["image"]
    for f in range(F):
        pf = p.astype(np.float64).copy()
        for t in range(f + 1):
            d = res[t].astype(np.float64)
            pf[0:3] += d[0:3]
            pf[10] += d[7]
            pf[3:6] += d[8:11]
            pf[11:] += d[11:]
            a = Rotation.from_quat(np.stack([d[4], d[5], d[6], d[3]], 1))
            b = Rotation.from_quat(np.stack([pf[7], pf[8], pf[9], pf[6]], 1))
            ab = (a * b).as_quat()  # unit quaternion of R(dq) R(q); the scale of q does not matter
            pf[6:10] = np.stack([ab[:, 3], ab[:, 0], ab[:, 1], ab[:, 2]])
        # The oracle composes in FP64 from float32 inputs; the composed params are handed to the
        # plain render in FP64 via a float32 round trip, so compare away from ambiguous pixels.
        st1 = oracle.Settings(48, 32, 1, (n,))
        ref = oracle.render(st1, pf.astype(np.float32), cams1, variants=True)
        ok = ref["nvar"][:, 0] == 0
        diff = np.abs(r[f * 2:(f + 1) * 2, 0] - ref["image"][:, 0]).max(axis=1)
        assert ok.mean() > 0.95
        assert diff[ok].max() < 1e-4


# ------------------------------------------------ order, near plane, ambiguity
def _pair_image(p, st, cam, px, py):
    r = oracle.render(st, p, cam, variants=True)
    return r["image"][0, 0, :, py, px], r["nvar"][0, 0, py, px]


def test_equal_depth_keys_composite_in_index_order():
    """Eq. 2 composites N ordered Gaussians. Reading: the order key is the float32 rounding of the
    exact camera depth, equal keys in index order. A camera turned by 1e-4 rad about y gives
    depth t_z = z - 1e-4 x, so a Gaussian at x = 1e-3 sits 1e-7 nearer than one at x = 0 with
    the same z = 3, and both depths round to the key 3.0f: the lower index is in front even
    where it is the deeper one. The two-layer closed form fixes the colour."""
    th = 1e-4
    cam = synth.identity_camera(W, H, FOC)[None].copy()
    cam[0, 0:3] = [math.cos(th), 0.0, math.sin(th)]
    cam[0, 8:11] = [-math.sin(th), 0.0, math.cos(th)]
    items = [([0, 0, 3.0], [math.log(0.2)] * 3, [1, 0, 0, 0], logit(0.6), [0.9, 0.1, 0.2]),
             ([1e-3, 0, 3.0], [math.log(0.2)] * 3, [1, 0, 0, 0], logit(0.5), [0.1, 0.7, 0.9])]
    st = oracle.Settings(W, H, 0, (2,), dilation=0.0)
    px, py = W // 2, H // 2
    for order in ([0, 1], [1, 0]):
        p = _stack([items[k] for k in order])
        pr = oracle.project(st, p, cam)[0]
        assert pr[0, 1] != pr[1, 1] and np.float32(pr[0, 1]) == np.float32(pr[1, 1]) == np.float32(3.0)
        c, nv = _pair_image(p, st, cam, px, py)
        a = []
        for k in range(2):
            dx, dy = px + 0.5 - pr[k, 2], py + 0.5 - pr[k, 3]
            g = math.exp(-0.5 * (pr[k, 7] * dx * dx + 2 * pr[k, 8] * dx * dy + pr[k, 9] * dy * dy))
            a.append(min(f32(0.99), pr[k, 10] * g))
        exp = pr[0, 11:14] * a[0] + pr[1, 11:14] * a[1] * (1 - a[0])
        np.testing.assert_allclose(c, exp, atol=1e-12)
        assert nv == 0


def test_near_plane_cull_is_exact_and_a_tie_is_explored():
    """A Gaussian with depth one float32 step beyond the near plane is rendered; one exactly on
    it is culled (t_z <= near), and because a depth that equals near cannot be settled by an
    evaluation with rounding error, the oracle also offers the outcome that keeps it."""
    near = np.float32(0.2)
    st = oracle.Settings(W, H, 0, (1,), near_plane=float(near), dilation=0.0)
    for z, culled in ((float(np.nextafter(near, np.float32(1.0))), False), (float(near), True)):
        p = scene([[0, 0, z]], [[math.log(0.002)] * 3], [[1, 0, 0, 0]], [logit(0.7)], [[0.8, 0.3, 0.5]])
        pr = oracle.project(st, p, cam0())[0]
        assert (pr[0, 0] == 0) == culled
        r = oracle.render(st, p, cam0(), variants=True)
        c = r["image"][0, 0, :, H // 2, W // 2]
        nv = r["nvar"][0, 0, H // 2, W // 2]
        if culled:
            assert np.all(c == 0.0) and nv == 2
            alts = r["var"][0, 0, H // 2, W // 2, :2]
            assert np.any(np.all(alts == 0.0, axis=1)) and np.any(alts.max(axis=1) > 0.1)
        else:
            assert c.max() > 0.1 and nv == 0


def test_alpha_cut_inside_its_band_offers_both_outcomes():
    """A candidate whose o G is within the float32 accuracy band of alpha_min is explored both
    ways (kept and cut); one well outside the band is not."""
    amin = f32(1.0 / 255.0)
    x = 0.5 * 3.0 / FOC  # projects to the centre of pixel (W/2, H/2): G = 1 there
    for rel, amb in ((2e-7, True), (1e-3, False)):
        o = amin * (1.0 + rel)
        p = scene([[x, x, 3.0]], [[math.log(0.05)] * 3], [[1, 0, 0, 0]], [logit(o)], [[0.8, 0.3, 0.5]])
        st = oracle.Settings(W, H, 0, (1,), dilation=0.0)
        pr = oracle.project(st, p, cam0())[0]
        assert pr[0, 2] == W // 2 + 0.5 and pr[0, 3] == H // 2 + 0.5
        assert abs(pr[0, 10] / amin - 1.0) < max(2 * rel, 5e-7)  # the float32 logit keeps o near the target
        r = oracle.render(st, p, cam0(), variants=True)
        nv = r["nvar"][0, 0, H // 2, W // 2]  # the mean sits on this pixel centre: G = 1
        if amb:
            assert nv == 2
            alts = r["var"][0, 0, H // 2, W // 2, :2]
            np.testing.assert_allclose(np.sort(alts[:, 0]), [0.0, pr[0, 11] * pr[0, 10]], atol=1e-15)
        else:
            assert nv == 0


def test_transmittance_stop_inside_its_band_offers_both_outcomes():
    """Two clamped layers (alpha = 0.99f each) leave T' = (1 - 0.99f)^2. With t_stop set to the
    float32 nearest T', the stop test is inside the accuracy band of the product: the oracle
    offers the colour with and without the second layer. With t_stop = 1e-4 it is settled."""
    items = [_big(2.0, 0.9995, [0.8, 0.1, 0.3]), _big(3.0, 0.9995, [0.2, 0.9, 0.5])]
    p = _stack(items)
    one_minus = 1.0 - f32(0.99)
    T2 = one_minus * one_minus
    for t_stop, amb in ((f32(T2), True), (1e-4, False)):
        st = oracle.Settings(W, H, 0, (2,), t_stop=t_stop)
        pr = oracle.project(st, p, cam0())[0]
        r = oracle.render(st, p, cam0(), variants=True)
        nv = r["nvar"][0, 0, H // 2, W // 2]
        if amb:
            assert nv == 2
            alts = np.sort(r["var"][0, 0, H // 2, W // 2, :2, 0])
            one = f32(0.99) * pr[0, 11]
            np.testing.assert_allclose(alts, [one, one + f32(0.99) * one_minus * pr[1, 11]], atol=1e-12)
        else:
            assert nv == 0
            assert r["ncontrib"][0, 0, H // 2, W // 2] == 1


def test_non_finite_and_zero_quaternion_gaussians_are_culled():
    """Reading: a Gaussian with a zero quaternion or any non-finite parameter is culled: the image
    equals the render without it and its gradient is zero."""
    w = synth.config_plain_forward(seed=13, n=120, width=40, height=32)
    cams = synth.identity_camera(40, 32, 40.0)[None]
    extra = w.params[:, :6].copy()
    for k, ch in enumerate([0, 4, 7, 10, 12]):
        extra[ch, k] = np.nan
    extra[6:10, 5] = 0.0
    p = np.ascontiguousarray(np.concatenate([w.params, extra], axis=1))
    st = oracle.Settings(40, 32, 0, (126,))
    a = oracle.render(st, p, cams)["image"]
    b = oracle.render(oracle.Settings(40, 32, 0, (120,)), w.params, cams)["image"]
    assert np.array_equal(a, b)
    dp, _, _ = oracle.backward(st, p, cams, np.random.default_rng(5).standard_normal(a.shape))
    assert np.all(dp[:, 120:] == 0.0) and np.isfinite(dp).all()
