"""hipGraph capture of the whole forward + fused-L1 backward step: every replay (with eager work
and synchronisations in between) reproduces the eager result."""
import numpy as np
import pytest
import torch

import synth
from parity import atomic_order_close, gpu_settings

pytestmark = pytest.mark.gpu


def test_graph_replays_match_eager():
    print("\n[case] graph capture of forward + backward, 3 replays", flush=True)
    from paper_2509_17513_amd import Workspace, render_backward, render_forward
    dev = torch.device("cuda:0")
    n = 3000
    p = synth.cube_scene(n, 81, 3)
    cams = synth.ring_cameras([0, 4, 9], 24, 4.0, 160, 96)
    w = synth.Workload("g", p, cams, 160, 96, 3, synth.nested_levels(n), synth.paper_level_weights(6),
                       target=synth.target_images(3, 160, 96, 82))
    st = gpu_settings(w)
    pt, ct, tt = (torch.from_numpy(a).to(dev) for a in (w.params, w.cams, w.target))
    img, ws = render_forward(st, pt, ct)  # sizes the workspace
    dp_ref, _ = render_backward(st, pt, ct, ws, image=img, target=tt)
    img_ref = img.clone()
    torch.cuda.synchronize()

    dp = torch.zeros_like(pt)
    loss = torch.zeros(1, device=dev)

    def step():
        dp.zero_()
        loss.zero_()
        render_forward(st, pt, ct, ws=ws, image=img, check_overflow=False)
        render_backward(st, pt, ct, ws, image=img, target=tt, d_params=dp, loss=loss)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    other_ws = Workspace(st, n, 1, 3, dev)
    for r in range(3):
        img.fill_(-1.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, img_ref), r
        ok, worst = atomic_order_close(dp.cpu().numpy(), dp_ref.cpu().numpy())
        print(f"replay {r}: gradients within {worst:.3f} of the atomic-order bar", flush=True)
        assert ok, (r, worst)
        assert loss.item() > 0
        # eager work on another workspace between replays
        render_forward(st, pt, ct, ws=other_ws)
        torch.cuda.synchronize()


def test_graph_replayed_step_matches_the_oracle():
    print("\n[case] captured forward + backward replayed 3 times, each replay against the FP64 oracle", flush=True)
    import oracle
    from parity import grad_mismatch, image_mismatch, l1_dimage, oracle_settings, param_groups
    from paper_2509_17513_amd import render_backward, render_forward
    dev = torch.device("cuda:0")
    n = 2500
    p = synth.cube_scene(n, 85, 3)
    cams = synth.ring_cameras([2, 11], 24, 4.0, 144, 96)
    w = synth.Workload("g", p, cams, 144, 96, 3, synth.nested_levels(n), synth.paper_level_weights(6),
                       target=synth.target_images(2, 144, 96, 86))
    st = gpu_settings(w)
    ost = oracle_settings(w)
    ref = oracle.render(ost, w.params, w.cams, variants=True)
    dimg = l1_dimage(ref, w.target, w.level_weights)
    dp_ref, _, _ = oracle.backward(ost, w.params, w.cams, dimg)
    pt, ct = (torch.from_numpy(a).to(dev) for a in (w.params, w.cams))
    img, ws = render_forward(st, pt, ct)  # sizes the workspace
    d_image = torch.from_numpy(dimg.astype(np.float32).reshape(img.shape)).to(dev)
    dp = torch.zeros_like(pt)

    def step():
        dp.zero_()
        render_forward(st, pt, ct, ws=ws, image=img, check_overflow=False)
        render_backward(st, pt, ct, ws, image=img, d_image=d_image, d_params=dp)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for r in range(3):
        img.fill_(-1.0)
        dp.fill_(123.0)
        g.replay()
        torch.cuda.synchronize()
        gi = img.cpu().numpy().reshape(ref["image"].shape)
        bad, amb, excl, err = image_mismatch(gi, ref)
        gb, worst = grad_mismatch(dp.cpu().numpy().astype(np.float64), dp_ref, param_groups(3))
        print(f"replay {r}: image bad={bad} ambiguous={amb} max_err={err:.3g}; grad bad={gb} worst={worst:.3g}",
              flush=True)
        assert bad == 0 and gb == 0
        render_forward(st, pt, ct)  # eager work between replays
        torch.cuda.synchronize()


def test_captured_joint_training_steps_match_eager_steps():
    print("\n[case] joint training (render + learned rate + Adam): captured replays vs eager steps", flush=True)
    from paper_2509_17513_amd import RenderSettings, render_forward
    from paper_2509_17513_amd.train import JointTrainer, RateModel
    dev = torch.device("cuda:0")
    n, W, H = 6000, 160, 96
    cams = torch.from_numpy(synth.ring_cameras([0, 8, 16], 24, 4.0, W, H)).to(dev)
    teacher = torch.from_numpy(synth.cube_scene(n, 1093, 3)).to(dev)
    timg, _ = render_forward(RenderSettings(W, H, 3, (n,), (1.0,)), teacher, cams)
    targets = timg[0, :, 0].contiguous()
    p0 = synth.cube_scene(n, 93, 3)
    st = RenderSettings(W, H, 3, tuple(synth.nested_levels(n)), tuple(synth.paper_level_weights(6)))

    def trainer():
        p = torch.from_numpy(p0.copy()).to(dev)
        return JointTrainer(p, cams, targets, st, RateModel(56, dev, seed=3, attrs=p[3:59]), lambda_rate=1e-3,
                            seed=3)

    K = 6
    ea, ca = trainer(), trainer()
    la, lc = [], []
    ea.step()
    ca.step()  # one eager step on both, then eager vs captured
    ca.capture()
    for _ in range(K):
        ea.step()
        la.append(float(ea.loss.item()))
        ca.step_graph()
        lc.append(float(ca.loss.item()))
    torch.cuda.synchronize()
    print("eager L1:   ", [round(x, 6) for x in la])
    print("captured L1:", [round(x, 6) for x in lc])
    assert int(ca.t_dev.item()) == ca.t == K + 1
    assert int(ca.off_dev.item()) == (K + 1) * 56 * n
    np.testing.assert_allclose(lc, la, rtol=1e-4)
    # float atomics make the two runs' gradients differ in the last bits; Adam moves a parameter by
    # at most about its learning rate per step, so the runs stay within K learning rates
    pa, pc = ea.p.cpu().numpy(), ca.p.cpu().numpy()
    lr = ea.lrs
    for lo, hi, r in ((0, 3, lr.mean), (3, 6, lr.log_scale), (6, 10, lr.quat), (10, 11, lr.logit),
                      (11, 14, lr.sh_dc), (14, 59, lr.sh_rest)):
        d = np.abs(pa[lo:hi] - pc[lo:hi])
        assert d.max() <= 2 * K * r, (lo, hi, d.max())
        assert np.median(d) <= 1e-3 * K * r, (lo, hi, np.median(d))
    np.testing.assert_allclose(ca.rate.w.cpu().numpy(), ea.rate.w.cpu().numpy(), atol=2 * K * lr.mlp)
