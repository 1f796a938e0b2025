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
