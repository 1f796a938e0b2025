"""Joint training on the GPU kernels (render forward/backward + learned rate + Adam), and what
the trained rate network gains over the method without it.

A student scene is fitted to renders of a seeded teacher scene (all views and six nested layers
at once). Checks: the layer-weighted L1 falls; the trained MLP's evaluation-mode rate is within 2%
of the empirical-histogram rate of the final attributes, on either side (the histogram rate
conditioned on layer x position octant is reported beside it, as the rate a context could reach);
the MLP's estimate error is no worse than a context-free Laplace fit and it
strictly gains on the attributes the significance ordering makes layer-dependent (scales,
opacity); and training with the rate term (lambda_rate > 0) cuts the histogram rate relative to
lambda_rate = 0 at a small, reported L1 increase.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _setup(lam, seed=91, n=20000, W=240, H=136, views=(0, 6, 12, 18)):
    from paper_2509_17513_amd import RenderSettings, render_forward
    from paper_2509_17513_amd.train import JointTrainer, RateModel
    dev = torch.device("cuda:0")
    teacher = torch.from_numpy(synth.cube_scene(n, seed + 1000, 3)).to(dev)
    cams = torch.from_numpy(synth.ring_cameras(list(views), 24, 4.0, W, H)).to(dev)
    st1 = RenderSettings(W, H, 3, (n,), (1.0,))
    timg, _ = render_forward(st1, teacher, cams)
    targets = timg[0, :, 0].contiguous()  # [V][3][H][W]
    # the hierarchy: Gaussians in decreasing significance (ordered by the oracle's ranking)
    from oracle.bitstream import significance_order
    p_host = synth.cube_scene(n, seed, 3)
    p_host = synth.reorder(p_host, significance_order(p_host))
    p = torch.from_numpy(p_host).to(dev)
    lv = synth.nested_levels(n)
    st = RenderSettings(W, H, 3, tuple(lv), tuple(synth.paper_level_weights(6)))
    rate = RateModel(56, dev, seed=seed, attrs=p[3:])
    return JointTrainer(p, cams, targets, st, rate, lambda_rate=lam, extent=1.0, seed=seed)


def _train(tr, steps):
    losses = []
    for t in range(steps):
        tr.step(check_overflow=(t == 0))
        if t % 10 == 0 or t == steps - 1:
            losses.append(float(tr.loss.item()))
    return losses


def test_joint_training_and_rate_network_gain():
    print("\n[case] joint training lambda_rate = 0 and > 0, 20k Gaussians, 4 views 240x136", flush=True)
    from oracle.rate import gaussian_fit_bits, laplace_fit_bits, layer_of
    steps = 120
    tr0 = _setup(0.0)
    l0 = _train(tr0, steps)
    print("L1 (lambda_rate=0):", [round(x, 5) for x in l0], flush=True)
    assert l0[-1] < 0.9 * l0[0]
    mlp, hist = tr0.eval_rate()
    attrs = tr0.p[3:59].cpu().numpy()
    lap = laplace_fit_bits(attrs, 1 / 64)
    gau = gaussian_fit_bits(attrs, 1 / 64)
    R_mlp, R_hist, R_lap, R_gau = mlp.sum(), hist.sum(), lap.sum(), gau.sum()
    from oracle.rate import bucketed_hist_bits, layer_octant_bucket
    n = attrs.shape[1]
    R_bkt = bucketed_hist_bits(attrs, 1 / 64, layer_octant_bucket(tr0.p[0:3].cpu().numpy(),
                                                                  layer_of(n, tr0.st.level_counts))).sum()
    print(f"bits: mlp {R_mlp:.0f} hist {R_hist:.0f} layer-x-octant hist {R_bkt:.0f} laplace-fit {R_lap:.0f} "
          f"gaussian-fit {R_gau:.0f}; mlp vs hist {(R_mlp - R_hist) / R_hist:+.4f}", flush=True)
    # the judge, two-sided: within 2% of the histogram rate of the final attributes
    assert abs(R_mlp - R_hist) <= 0.02 * R_hist
    e_mlp = abs(R_mlp - R_hist) / R_hist
    e_lap = abs(R_lap - R_hist) / R_hist
    assert e_mlp <= e_lap + 1e-3
    # scales and opacity are ordered by significance, so the layer feature of the context is informative
    gain = lap[[0, 1, 2, 7]] - mlp[[0, 1, 2, 7]]
    print("context gain on log-scale x/y/z and opacity (bits):", np.round(gain, 1), flush=True)
    assert gain.sum() > 0

    tr1 = _setup(3e-3)
    l1 = _train(tr1, steps)
    _, hist1 = tr1.eval_rate()
    print(f"lambda_rate=3e-3: L1 {l1[-1]:.5f} (vs {l0[-1]:.5f}); histogram bits {hist1.sum():.0f} "
          f"(vs {R_hist:.0f}, {(hist1.sum() - R_hist) / R_hist:+.4f})", flush=True)
    assert hist1.sum() < R_hist
    assert l1[-1] < 1.25 * l0[-1]


def _dssim(tr):
    """Layer-weighted D-SSIM of the trainer's current render (gs_color_loss, lambda_ssim = 1)."""
    from paper_2509_17513_amd import color_loss, render_forward
    render_forward(tr.st, tr.p, tr.cams, ws=tr.ws, image=tr.img)
    v = torch.zeros(1, device=tr.p.device)
    color_loss(tr.st, tr.img, tr.tgt, 1.0, loss=v, grad=False)
    return float(v.item())


def test_training_with_dssim_term():
    print("\n[case] keyframe training with the D-SSIM term (lambda_ssim = 0.2) vs without", flush=True)
    from paper_2509_17513_amd.train import JointTrainer
    res = {}
    for lam in (0.0, 0.2):
        tr = _setup(0.0)
        tr = JointTrainer(tr.p, tr.cams, tr.tgt, tr.st, None, lambda_ssim=lam, seed=91)
        d0 = _dssim(tr)
        losses = _train(tr, 60)
        res[lam] = (losses, d0, _dssim(tr))
        print(f"lambda_ssim={lam}: loss {[round(x, 5) for x in losses]}, D-SSIM {d0:.5f} -> {res[lam][2]:.5f}",
              flush=True)
    losses, d0, d1 = res[0.2]
    assert losses[-1] < 0.9 * losses[0]
    assert d1 < d0
    print(f"D-SSIM after 60 steps: {res[0.2][2]:.5f} with the term, {res[0.0][2]:.5f} without", flush=True)


def test_rigid_phase_recovers_a_translation():
    """Inter-frame rigid phase end to end (motion module -> render with residuals -> L1 backward to
    the residuals -> motion backward -> Adam): the views of the keyframe moved by a known
    translation are fitted, so the loss falls and the predicted translations point along it."""
    print("\n[case] rigid phase: 20k Gaussians, 4 views 240x136, target = keyframe moved by t", flush=True)
    from paper_2509_17513_amd import RenderSettings, render_forward
    from paper_2509_17513_amd.motion import sizes
    from paper_2509_17513_amd.train import RigidTrainer
    from oracle import motion as M
    dev = torch.device("cuda:0")
    n, W, H = 20000, 240, 136
    key = synth.cube_scene(n, 61, 1)
    shift = np.array([0.06, -0.03, 0.02], np.float32)
    moved = key.copy()
    moved[0:3] += shift[:, None]
    cams = torch.from_numpy(synth.ring_cameras([0, 6, 12, 18], 24, 4.0, W, H)).to(dev)
    st1 = RenderSettings(W, H, 1, (n,), (1.0,))
    timg, _ = render_forward(st1, torch.from_numpy(moved).to(dev), cams)
    targets = timg[0, :, 0].contiguous()
    st = RenderSettings(W, H, 1, (n // 2, n), (0.5, 1.0))
    nt, nw = sizes()
    shapes = [s for out in (3, 4) for s in M.head_sizes(out)]
    table, w = synth.motion_params(62, nt, shapes, table_scale=1e-4)
    tr = RigidTrainer(torch.from_numpy(key).to(dev), cams, targets, st, (-1.2, -1.2, -1.2), (1.2, 1.2, 1.2),
                      torch.from_numpy(table).to(dev), torch.from_numpy(w * 0.1).to(dev))
    losses = []
    for t in range(150):
        tr.step(check_overflow=(t == 0))
        if t % 25 == 0 or t == 149:
            losses.append(float(tr.loss.item()))
    mean_t = tr.translation().mean(dim=1).cpu().numpy()
    print(f"loss {[round(x, 5) for x in losses]}; mean predicted translation {np.round(mean_t, 4)} vs {shift}",
          flush=True)
    assert losses[-1] < 0.67 * losses[0]
    assert float(mean_t @ shift) > 0.5 * float(shift @ shift)


def test_keyframe_training_with_the_kde_rate():
    """The paper's keyframe objective with its own rate (Sec. 3.3): sum_l lambda^l (L1^l +
    lambda_rate KDE-rate^l). Training with the rate term cuts the histogram rate of the attributes
    relative to lambda_rate = 0 at a small L1 increase."""
    print("\n[case] keyframe training with the KDE rate, lambda_rate 0 vs 3e-3", flush=True)
    from paper_2509_17513_amd.train import JointTrainer
    res = {}
    for lam in (0.0, 3e-3):
        base = _setup(0.0)
        tr = JointTrainer(base.p, base.cams, base.tgt, base.st, None, lambda_rate=lam, seed=91, kde_rate=True)
        losses = _train(tr, 120)
        res[lam] = (losses[-1], tr.histogram_rate().sum(), float(tr.kde_loss.item()))
        print(f"lambda_rate={lam}: L1 {losses[0]:.5f} -> {losses[-1]:.5f}, histogram bits {res[lam][1]:.0f}, "
              f"KDE rate term {res[lam][2]:.4g}", flush=True)
    assert res[3e-3][1] < res[0.0][1]
    assert res[3e-3][0] < 1.25 * res[0.0][0]


def test_residual_phase_fits_and_the_rate_terms_shrink_residuals():
    """Inter-frame residual deformation (Sec. 3.2-3.3): targets are the keyframe with changed
    colours and opacities; training the residual rows fits them, and the Gaussian rate + temporal L1
    terms keep the residuals smaller than training without them."""
    print("\n[case] residual phase: 20k Gaussians SH 1, 4 views 240x136, lambda 0 vs (1e-4, 1e-3)", flush=True)
    from paper_2509_17513_amd import RenderSettings, render_forward
    from paper_2509_17513_amd.train import ResidualTrainer
    dev = torch.device("cuda:0")
    n, W, H = 20000, 240, 136
    key = synth.cube_scene(n, 71, 1)
    changed = key.copy()
    rng = np.random.default_rng(72)
    changed[11:14] += 0.15            # brighter base colour
    changed[10] += rng.normal(0, 0.3, n).astype(np.float32)  # opacity changes
    cams = torch.from_numpy(synth.ring_cameras([0, 6, 12, 18], 24, 4.0, W, H)).to(dev)
    timg, _ = render_forward(RenderSettings(W, H, 1, (n,), (1.0,)), torch.from_numpy(changed).to(dev), cams)
    targets = timg[0, :, 0].contiguous()
    st = RenderSettings(W, H, 1, (n // 2, n), (0.5, 1.0))
    C = key.shape[0]
    out = {}
    for lam_rate, lam_reg in ((0.0, 0.0), (1e-4, 1e-3)):
        res = torch.zeros((1, C, n), device=dev)
        res[0, 3] = 1.0  # identity rotation, no translation: the frame differs by the residual rows only
        tr = ResidualTrainer(torch.from_numpy(key).to(dev), res, cams, targets, st, lam_rate, lam_reg, lr=2e-2)
        losses = []
        for t in range(120):
            tr.step(check_overflow=(t == 0))
            if t % 30 == 0 or t == 119:
                losses.append(float(tr.loss.item()))
        out[(lam_rate, lam_reg)] = (losses, float(res[0, 7:].abs().sum().item()))
        print(f"lambda_rate={lam_rate} lambda_reg={lam_reg}: L1 {[round(x, 5) for x in losses]}, "
              f"sum |residual| {out[(lam_rate, lam_reg)][1]:.1f}", flush=True)
    free, reg = out[(0.0, 0.0)], out[(1e-4, 1e-3)]
    assert free[0][-1] < 0.7 * free[0][0] and reg[0][-1] < 0.8 * reg[0][0]
    assert reg[1] < free[1]


def test_trainer_grows_an_overflowing_pair_list_instead_of_training_on_a_stale_image():
    print("\n[case] joint training started with a pair list far too small: the trainer grows it", flush=True)
    tr = _setup(1e-3)
    ref = _setup(1e-3)
    tr.ws.allocate(4096)  # far fewer (tile, Gaussian) pairs than the scene needs
    cap0 = tr.ws.pair_capacity
    for _ in range(3):
        tr.step()
        ref.step()
    losses = float(tr.loss.item()), float(ref.loss.item())
    print(f"capacity {cap0} -> {tr.ws.pair_capacity}; loss {losses[0]:.6f} (vs {losses[1]:.6f} sized up front)",
          flush=True)
    assert tr.ws.pair_capacity > cap0
    assert losses[0] > 0.1 and abs(losses[0] - losses[1]) <= 1e-4 * losses[1]
