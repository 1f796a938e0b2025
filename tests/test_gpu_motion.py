"""GPU parity of the rigid-motion module (gs_motion_forward / gs_motion_backward through the C
ABI) against the FP64 oracle. FP32 sums of at most 64 terms of size ~1 (the MLPs) and float-atomic
sums over Gaussians (the table and weight gradients): outputs to 1e-5 (1 + |value|), each
gradient tensor to 1e-4 of its largest entry plus 1e-4 of the entry.

A ReLU whose pre-activation is within FP32 rounding of zero can take the other side on the GPU;
such a flip changes that Gaussian's gradient by about its own size, which is not rounding. So the
output gradient of every Gaussian with a pre-activation within 1e-4 of a kink (in FP64; ~2% of
them) is set to zero for both sides: its mask then does not matter."""
import numpy as np
import pytest
import torch

import synth
from oracle import motion as M

pytestmark = pytest.mark.gpu
LO, HI = (-1.0, -1.0, -1.0), (1.0, 1.0, 1.0)


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch.device("cuda:0")


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _inputs(n, seed, outside=True):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-1, 1, (3, n)).astype(np.float32)
    if outside:
        mu[:, :5] = [[1.5, -3, 0.2, 1.0, -1.0], [0.1, 0.0, 2.0, 1.0, -1.0], [0.3, 0.3, -9.0, 1.0, -1.0]]
    shapes = [s for out in (3, 4) for s in M.head_sizes(out)]
    table, w = synth.motion_params(seed, M.LEVELS * M.T * M.FEATS, shapes, table_scale=0.5)
    return mu, table, w


def _gpu(mu, table, w, d_out=None, rows=7):
    from paper_2509_17513_amd.motion import MotionModule
    dev = _dev()
    n = mu.shape[1]
    mm = MotionModule(n, LO, HI, dev)
    m, t, ww = (torch.from_numpy(a).to(dev) for a in (mu, table, w))
    out = torch.full((rows + 1, n), -7.0, device=dev)
    mm.forward(m, t, ww, out)
    res = {"out": out}
    if d_out is not None:
        dt = torch.zeros_like(t)
        dw = torch.zeros_like(ww)
        dy = torch.zeros((rows + 1, n), device=dev)
        dy[:7] = torch.from_numpy(d_out.astype(np.float32)).to(dev)
        mm.backward(m, t, ww, dy, dt, dw)
        res.update(dt=dt, dw=dw)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().astype(np.float64) for k, v in res.items()}


def _away_from_kinks(mu, table, w, d_out):
    near = M.min_preactivation(mu, LO, HI, table, w) < 1e-4
    d = d_out.copy()
    d[:, near] = 0.0
    print(f"{near.sum()} of {near.size} Gaussians near a ReLU kink: output gradient zeroed", flush=True)
    return d


def _close(got, ref, rel=1e-4):
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    bar = rel * scale + rel * np.abs(ref)
    return (err <= bar).all(), float((err / np.maximum(bar, 1e-300)).max())


def test_forward_and_backward_match_oracle():
    _case("motion module 4000 Gaussians (5 outside the box): forward, table and weight gradients")
    mu, table, w = _inputs(4000, 1)
    d_out = _away_from_kinks(mu, table, w, np.random.default_rng(2).normal(0, 1, (7, 4000)))
    g = _gpu(mu, table, w, d_out)
    ref = M.forward(mu, LO, HI, table, w)
    assert np.all(np.abs(g["out"][:7] - ref) <= 1e-5 * (1 + np.abs(ref)))
    assert np.all(g["out"][7] == -7.0)  # only rows 0..6 are written
    dt, dw = M.backward(mu, LO, HI, table, w, d_out)
    ok_t, wt = _close(g["dt"], dt)
    sizes = [int(np.prod(s)) for out in (3, 4) for s in M.head_sizes(out)]
    bounds = np.cumsum([0] + sizes)
    worst = 0.0
    for k in range(len(sizes)):
        ok, r = _close(g["dw"][bounds[k]:bounds[k + 1]], dw[bounds[k]:bounds[k + 1]])
        worst = max(worst, r)
        assert ok, (k, r)
    print(f"table gradient within {wt:.3f} of its bar, weights within {worst:.3f}")
    assert ok_t, wt


def test_zero_weights_give_the_identity():
    _case("motion module with zero weights: no translation, identity rotation")
    mu, table, w = _inputs(300, 3)
    g = _gpu(mu, table, np.zeros_like(w))
    assert np.all(g["out"][0:3] == 0) and np.all(g["out"][3] == 1) and np.all(g["out"][4:7] == 0)


@pytest.mark.parametrize("n", [1, 255, 257])
def test_small_counts(n):
    _case(f"motion module n={n}")
    mu, table, w = _inputs(n, 10 + n, outside=n >= 5)
    d_out = _away_from_kinks(mu, table, w, np.random.default_rng(n).normal(0, 1, (7, n)))
    g = _gpu(mu, table, w, d_out)
    ref = M.forward(mu, LO, HI, table, w)
    assert np.all(np.abs(g["out"][:7] - ref) <= 1e-5 * (1 + np.abs(ref)))
    dt, dw = M.backward(mu, LO, HI, table, w, d_out)
    assert _close(g["dt"], dt)[0] and _close(g["dw"], dw)[0]


def test_fullsize_300k():
    _case("motion module 300k Gaussians: forward and gradients against the oracle")
    n = 300_000
    mu, table, w = _inputs(n, 4, outside=False)
    d_out = _away_from_kinks(mu, table, w, np.random.default_rng(5).normal(0, 1e-3, (7, n)))
    g = _gpu(mu, table, w, d_out)
    ref = M.forward(mu, LO, HI, table, w)
    assert np.all(np.abs(g["out"][:7] - ref) <= 1e-5 * (1 + np.abs(ref)))
    dt, dw = M.backward(mu, LO, HI, table, w, d_out)
    ok_t, wt = _close(g["dt"], dt)
    ok_w, ww = _close(g["dw"], dw)
    print(f"table gradient within {wt:.3f} of its bar, weights within {ww:.3f}")
    assert ok_t and ok_w
