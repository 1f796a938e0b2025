"""Parity at the workloads' full sizes, in the launch configuration the benchmark times (all
views, frames and layers in one call), on outputs the oracle can compute one by one: sampled
pixels of every view and layer, gradients of a loss restricted to pixel windows, FP64 finite
differences of sampled parameters, and sampled rate symbols.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import rate
from parity import (ambiguity_report, gpu_settings, grad_mismatch, image_mismatch, l1_dimage, oracle_settings,
                    param_groups)

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _forward(w, bwd_pixels=0):
    from paper_2509_17513_amd import render_forward
    dev = torch.device("cuda:0")
    st = gpu_settings(w, bwd_pixels=bwd_pixels)
    p = torch.from_numpy(w.params).to(dev)
    c = torch.from_numpy(w.cams).to(dev)
    r = None if w.residuals is None else torch.from_numpy(w.residuals).to(dev)
    img, ws = render_forward(st, p, c, w.n_frames, r)
    torch.cuda.synchronize()
    return img, ws, (p, c, r, st)


def _sample_pixels(w, count, seed):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(w.width * w.height, count, replace=False)).astype(np.int64)


def _gather(img, pix, w):
    a = img.reshape(img.shape[0] * img.shape[1], img.shape[2], 3, w.height * w.width)
    return a[..., torch.from_numpy(pix).to(img.device)].cpu().numpy()


def test_batched_300k_24views_sampled_pixels():
    _case("300k Gaussians, 24 views 960x540, 6 layers: 400 sampled pixels x every view x every layer")
    w = synth.config_batched()
    img, _, _ = _forward(w)
    pix = _sample_pixels(w, 400, 101)
    ref = oracle.render(oracle_settings(w), w.params, w.cams, sample=pix, variants=True)
    gi = _gather(img, pix, w)
    bad, amb, excl, err = image_mismatch(gi, ref)
    rep = ambiguity_report(gi, ref)
    print(f"bad={bad} ambiguous={amb} excluded={excl} of {ref['nvar'].size}; max_err={err:.3g}; {rep}")
    assert bad == 0
    assert excl <= 1e-4 * ref["nvar"].size
    # the oracle's float32 accuracy bands flag about 0.9% of these pixel-levels (half of them with
    # alternatives farther apart than the tolerance); these bounds catch a band that widens
    assert rep["ambiguous"] <= 0.015 * rep["total"] and rep["material"] <= 0.006 * rep["total"]


def _window_dimage(w, img, views, x0, y0, size, seed):
    """L1-like weights (fixed random signs, layer weights / (3HW)) inside a window of the given
    views, zero elsewhere: one device tensor for the GPU, one float64 array for the oracle."""
    rng = np.random.default_rng(seed)
    B, L = w.cams.shape[0], len(w.level_counts)
    d = np.zeros((B, L, 3, w.height, w.width))
    lw = np.asarray(w.level_weights).reshape(L, 1, 1, 1)
    for v in views:
        d[v, :, :, y0:y0 + size, x0:x0 + size] = lw * rng.choice([-1.0, 1.0], (L, 3, size, size)) / (
            3.0 * w.width * w.height)
    return d


@pytest.mark.parametrize("bwd_pixels", [1, 2])
def test_batched_300k_windowed_gradients_match_oracle(bwd_pixels):
    _case(f"300k Gaussians, 3 ring views 960x540, 6 layers: gradient of a windowed loss vs oracle "
          f"({bwd_pixels} pixel(s) per lane)")
    from paper_2509_17513_amd import render_backward
    w = synth.config_batched(view_indices=(0, 8, 16))
    img, ws, (p, c, r, st) = _forward(w, bwd_pixels)
    ost = oracle_settings(w)
    d = _window_dimage(w, img, (0, 2), 440, 230, 64, 102)
    # pixel-levels whose FP32 / FP64 decisions may differ carry no weight on either side
    pix = np.array([(y * w.width + x) for y in range(230, 294) for x in range(440, 504)], np.int64)
    ref = oracle.render(ost, w.params, w.cams, sample=pix, variants=True)
    amb = ref["nvar"] != 0  # [B][L][S]
    dflat = d.reshape(d.shape[0], d.shape[1], 3, -1)
    for b in range(d.shape[0]):
        for l in range(d.shape[1]):
            dflat[b, l][:, pix[amb[b, l]]] = 0.0
    dp_ref, _, _ = oracle.backward(ost, w.params, w.cams, d)
    dimg = torch.from_numpy(d.astype(np.float32).reshape(img.shape)).to(p.device)
    dp, _ = render_backward(st, p, c, ws, image=img, d_image=dimg)
    torch.cuda.synchronize()
    touched = np.abs(dp_ref).sum(axis=0) > 0
    print(f"Gaussians with gradient: {touched.sum()}")
    bad, worst = grad_mismatch(dp.cpu().numpy()[:, touched].astype(np.float64), dp_ref[:, touched],
                               param_groups(w.sh_degree))
    print(f"grad bad={bad} of {touched.sum() * 59} worst_ratio={worst:.3g}")
    assert bad == 0
    assert np.all(dp.cpu().numpy()[:, ~touched] == 0)


def _fd_strata(pr, touched, w, rng, per=64):
    """256 Gaussians in four strata of 64: front (smallest depth), deep (largest depth that still
    gets a gradient), edge (footprint crossing the image border) and near-cutoff (lowest opacity,
    so that most of the footprint lies near the 1/255 cut)."""
    idx = np.nonzero(touched)[0]
    tz, mx, my, rad, o = pr[idx, 1], pr[idx, 2], pr[idx, 3], pr[idx, 14], pr[idx, 10]
    taken = np.zeros(len(idx), bool)
    out = {}

    def pick(name, order):
        sel = [k for k in order if not taken[k]][:per]
        taken[sel] = True
        out[name] = idx[sel]

    pick("front", np.argsort(tz, kind="stable"))
    pick("deep", np.argsort(-tz, kind="stable"))
    edge = np.nonzero((mx - rad < 0) | (mx + rad > w.width) | (my - rad < 0) | (my + rad > w.height))[0]
    pick("edge", rng.permutation(edge))
    pick("near_cutoff", np.argsort(o, kind="stable"))
    return out


def test_fwd_bwd_200k_1280x720_against_finite_differences():
    _case("200k Gaussians SH3 1280x720, L1 loss: GPU gradients vs the oracle's analytic backward (all "
          "11.8M) and vs FP64 central differences (256 stratified Gaussians x 59 + 1000 random)")
    from paper_2509_17513_amd import render_backward
    w = synth.config_forward_backward()
    img, ws, (p, c, r, st) = _forward(w)
    ost = oracle_settings(w)
    ref = oracle.render(ost, w.params, w.cams, variants=True)
    gi_img = img.cpu().numpy().reshape(ref["image"].shape)
    bad, amb, excl, err = image_mismatch(gi_img, ref)
    print(f"image bad={bad} ambiguous={amb} excluded={excl} max_err={err:.3g}; {ambiguity_report(gi_img, ref)}",
          flush=True)
    assert bad == 0
    d = l1_dimage(ref, w.target, w.level_weights).astype(np.float32)
    dimg = torch.from_numpy(d.reshape(img.shape)).to(p.device)
    dp, _ = render_backward(st, p, c, ws, image=img, d_image=dimg)
    torch.cuda.synchronize()
    g = dp.cpu().numpy().astype(np.float64)
    d = d.astype(np.float64)
    dp_ref, _, _ = oracle.backward(ost, w.params, w.cams, d)
    groups = param_groups(w.sh_degree)
    bad, worst = grad_mismatch(g, dp_ref, groups)
    touched = np.abs(dp_ref).sum(axis=0) > 0
    print(f"analytic: bad={bad} of {g.size} worst_ratio={worst:.3g}; Gaussians with gradient {touched.sum()}",
          flush=True)
    assert bad == 0
    assert np.all(g[:, ~touched] == 0)
    # finite differences of the same linear functional sum(d * image)
    pr = oracle.project(ost, w.params, w.cams)[0]
    rng = np.random.default_rng(104)
    strata = _fd_strata(pr, touched, w, rng)
    C = w.params.shape[0]
    gi = np.concatenate([np.repeat(v, C) for v in strata.values()])
    ci = np.concatenate([np.tile(np.arange(C), len(v)) for v in strata.values()])
    rest = np.setdiff1d(np.nonzero(touched)[0], gi)
    gi = np.concatenate([gi, rng.choice(rest, 1000)]).astype(np.int32)
    ci = np.concatenate([ci, rng.integers(0, C, 1000)]).astype(np.int32)
    labels = np.concatenate([np.repeat(k, len(v) * C) for k, v in strata.items()] + [np.repeat("random", 1000)])
    fd, status, skipped = oracle.finite_differences(ost, w.params, w.cams, d, gi, ci, h=1e-5)
    assert np.all(status & 8 == 0)
    ok = (status & 4) == 0
    grp = np.zeros(C, int)
    for k, (lo, hi) in enumerate(groups):
        grp[lo:hi] = k
    # RMS of the oracle's gradient over the attribute group, over every Gaussian with a gradient
    rms = np.array([np.sqrt(np.mean(dp_ref[lo:hi][:, touched] ** 2)) for lo, hi in groups])[grp[ci]]
    got, ana = g[ci, gi], dp_ref[ci, gi]
    ratio = np.abs(got - fd) / (1e-3 * np.abs(fd) + 1e-3 * rms)
    rel = np.abs(got - fd) / np.maximum(np.abs(fd), 1e-300)
    big = ok & (np.abs(fd) >= rms)  # far above the float32 noise of a sum of per-pixel terms
    for k in list(strata) + ["random"]:
        m = labels == k
        print(f"  {k:12s} params={m.sum():5d} skipped={np.sum(m & ~ok):3d} one-sided={np.sum(m & (status & 1 > 0)):4d} "
              f"h/10={np.sum(m & (status & 2 > 0)):3d} worst_ratio={ratio[m & ok].max():.3g} "
              f"max_rel(|fd|>=rms)={rel[m & big].max() if np.any(m & big) else 0:.3g}")
    for k, (lo, hi) in enumerate(groups):
        m = (ci >= lo) & (ci < hi)
        print(f"  group {lo}-{hi}: params={m.sum()} skipped={np.sum(m & ~ok)}")
    print(f"FD checked={ok.sum()} of {len(ok)} worst_ratio={ratio[ok].max():.3g} "
          f"oracle analytic vs FD worst={np.max(np.abs(ana - fd)[ok] / (1e-3 * np.abs(fd) + 1e-3 * rms)[ok]):.3g}")
    assert np.all(ratio[ok] <= 1.0)
    assert np.all(rel[big] <= 1e-3)
    assert ok.mean() >= 0.98


def test_group_150k_10frames_8views_sampled():
    _case("150k Gaussians, 10 frames x 8 views 960x540 in one call: sampled pixels and residual gradients")
    from paper_2509_17513_amd import render_backward
    w = synth.config_group()
    img, ws, (p, c, r, st) = _forward(w)
    ost = oracle_settings(w)
    pix = _sample_pixels(w, 120, 105)
    ref = oracle.render(ost, w.params, w.cams, n_frames=w.n_frames, residuals=w.residuals, sample=pix,
                        variants=True)
    bad, amb, excl, err = image_mismatch(_gather(img, pix, w), ref)
    print(f"bad={bad} ambiguous={amb} excluded={excl} of {ref['nvar'].size}; max_err={err:.3g}")
    assert bad == 0
    # windowed loss in frames 0 and 9 (view 2): gradients to the keyframe and to every frame's residuals
    B = w.cams.shape[0]
    d = np.zeros((B, 1, 3, w.height, w.width))
    rng = np.random.default_rng(106)
    for b in (2, 9 * 8 + 2):
        d[b, 0, :, 250:290, 460:500] = rng.choice([-1.0, 1.0], (3, 40, 40)) / (3.0 * w.width * w.height)
    wpix = np.array([(y * w.width + x) for y in range(250, 290) for x in range(460, 500)], np.int64)
    refw = oracle.render(ost, w.params, w.cams, n_frames=w.n_frames, residuals=w.residuals, sample=wpix,
                         variants=True)
    df = d.reshape(B, 1, 3, -1)
    for b in range(B):
        df[b, 0][:, wpix[refw["nvar"][b, 0] != 0]] = 0.0
    dp_ref, dr_ref, _ = oracle.backward(ost, w.params, w.cams, d, n_frames=w.n_frames, residuals=w.residuals)
    dimg = torch.from_numpy(d.astype(np.float32).reshape(img.shape)).to(p.device)
    dp, dr = render_backward(st, p, c, ws, w.n_frames, r, image=img, d_image=dimg)
    torch.cuda.synchronize()
    touched = np.abs(dp_ref).sum(axis=0) > 0
    b1, w1 = grad_mismatch(dp.cpu().numpy()[:, touched].astype(np.float64), dp_ref[:, touched], param_groups(3))
    drn = dr.cpu().numpy().astype(np.float64)
    b2, w2 = grad_mismatch(drn[:, :, touched].transpose(1, 0, 2).reshape(8, -1),
                           dr_ref[:, :, touched].transpose(1, 0, 2).reshape(8, -1), [(0, 3), (3, 7), (7, 8)])
    print(f"touched={touched.sum()} params bad={b1} worst={w1:.3g}; residuals bad={b2} worst={w2:.3g}")
    assert b1 == 0 and b2 == 0


def test_rate_1M_x_56_histogram_and_sampled_symbols():
    _case("rate: 1M Gaussians x 56 attributes, histogram exact, MLP sampled symbols")
    import ctypes

    from paper_2509_17513_amd import _lib
    from paper_2509_17513_amd.train import RateModel, context, histogram_bits
    dev = torch.device("cuda:0")
    n = 1_000_000
    p_host = synth.cube_scene(n, 5, 3)
    p = torch.from_numpy(p_host).to(dev)
    attrs = p[3:59]
    hb = histogram_bits(attrs).cpu().numpy()
    np.testing.assert_allclose(hb, rate.hist_bits(p_host[3:59], 1 / 64), rtol=1e-12)
    lv = synth.nested_levels(n)
    lw = synth.paper_level_weights(6)
    rm = RateModel(56, dev, seed=5, attrs=attrs)
    ctx = context(p, 1.0, lv)
    sym = torch.zeros((56, n), dtype=torch.float32, device=dev)
    rm.reset()
    rm.run(ctypes.c_void_p(p.data_ptr() + 4 * 3 * n), n, ctx, 0, lv, lw, 1.0, grads=False, sym_bits=sym)
    torch.cuda.synchronize()
    cols = np.sort(np.random.default_rng(107).choice(n, 3000, replace=False))
    ctx_h = rate.bf16_bits_to_f64(ctx.cpu().numpy().view(np.uint16)[cols]).T
    ref_ctx = rate.context(p_host[0:3, cols], 1.0, rate.layer_of(n, lv)[cols])
    assert (ctx_h != ref_ctx).mean() < 1e-3
    wbits = rm.w16.cpu().numpy().view(np.uint16)
    bref = rm.b.cpu().numpy()
    out = rate.rate_model(p_host[3:59, cols], ref_ctx, wbits, bref, 1 / 64, mode=0, want_grad=False)
    got = sym.cpu().numpy()[:, cols]
    # per symbol: the oracle's bits from its own context; BF16 rounding flips allow 1e-2
    ref_sym = np.stack([rate.laplace_bits(np.rint(p_host[3 + a, cols].astype(np.float64) * 64) / 64,
                                          out["m"][a], out["b"][a], 1 / 64)[0] for a in range(56)])
    rel = np.abs(got - ref_sym) / np.maximum(ref_sym, 1.0)
    print(f"per-symbol rel err: median {np.median(rel):.2e} p99.9 {np.quantile(rel, 0.999):.2e}")
    assert np.quantile(rel, 0.999) < 1e-2
    tot = rm.bits.cpu().numpy()
    assert np.all(np.abs(tot - got.sum(axis=1) * n / len(cols)) < 0.05 * tot)
    del _lib
