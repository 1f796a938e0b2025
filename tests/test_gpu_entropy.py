"""GPU parity of the paper's entropy models (gs_entropy_model through the C ABI) against the
oracle: the KDE rate of keyframe attributes and the Gaussian rate with the temporal L1 term of
residual attributes.

Bars: the KDE's counts are binned in fixed point (2^-16 of a symbol) and the symbols may differ by
an FP32 rounding, so per-symbol bits agree to 1e-4 + 1e-5 bits (symbols whose probability is
within 1e-4 of the 1e-9 floor excepted), totals and loss to 1e-6 relative, and each (layer,
attribute) segment's gradient to 1e-3 of its largest value. The Gaussian model is evaluated in
FP64 from FP64 sums: bits to 1e-6, gradients to 1e-4 of the segment's largest.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import entropy as E

pytestmark = pytest.mark.gpu
Q = 1.0 / 64


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch.device("cuda:0")


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _run(attrs, kind, mode, lv, lw, lam=1.0, reg=0.0, seed=7, offset=11):
    from paper_2509_17513_amd.entropy import EntropyModel
    dev = _dev()
    A, n = attrs.shape
    em = EntropyModel(A, n, kind, dev, Q, lv, lw, lam, reg)
    at = torch.from_numpy(attrs).to(dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    sb = torch.empty_like(at)
    da = torch.zeros_like(at)
    bits = em.run(at, mode, seed, offset, loss=loss, sym_bits=sb, d_attrs=da).clone()
    torch.cuda.synchronize()
    return bits.cpu().numpy(), loss.item(), sb.cpu().numpy().astype(np.float64), da.cpu().numpy().astype(np.float64)


def _check(attrs, kind, mode, lv, lw, lam=1.0, reg=0.0, seed=7, offset=11):
    bits, loss, sym, grad = _run(attrs, kind, mode, lv, lw, lam, reg, seed, offset)
    rb, rl, rs, rg = E.entropy_model(attrs, Q, kind, mode, seed, offset, lv, lw, lam, reg)
    floor_bits = -np.log2(E.P_FLOOR)
    near_floor = np.abs(rs - floor_bits) < 2e-4 * floor_bits
    tol = (1e-4 + 1e-5 * rs) if kind == 0 else (1e-6 + 1e-7 * rs)
    bad = (np.abs(sym - rs) > tol) & ~near_floor
    assert not bad.any(), (np.argwhere(bad)[:5], sym[bad][:5], rs[bad][:5])
    assert np.allclose(bits, rb, rtol=1e-6, atol=1e-6)
    assert abs(loss - rl) <= 1e-6 * abs(rl) + 1e-9
    if mode == 1:
        bounds = [0] + list(lv)
        gt = 1e-3 if kind == 0 else 1e-4
        for l in range(len(lv)):
            for a in range(attrs.shape[0]):
                r = rg[a, bounds[l]:bounds[l + 1]]
                g = grad[a, bounds[l]:bounds[l + 1]]
                if r.size == 0:
                    continue
                scale = np.abs(r).max()
                ok = ~near_floor[a, bounds[l]:bounds[l + 1]]
                assert np.abs(g - r)[ok].max(initial=0.0) <= gt * scale + 1e-12, (l, a)
    else:
        assert not grad.any()
    print(f"bits {bits.sum():.1f} (oracle {rb.sum():.1f}), loss {loss:.6g} (oracle {rl:.6g}), "
          f"worst symbol {np.abs(sym - rs)[~near_floor].max():.2e} bits")


def _attrs(n, seed, A=6):
    p = synth.cube_scene(n, seed, 1)
    return np.ascontiguousarray(p[3:3 + A])  # log-scales, quaternion: irregular, layer-dependent


@pytest.mark.parametrize("mode", [0, 1])
def test_kde_matches_oracle(mode):
    _case(f"KDE rate, 6 attributes x 5000, layers 1000/2500/5000, mode {mode}")
    _check(_attrs(5000, 3), 0, mode, [1000, 2500, 5000], [0.5, 0.25, 1.0], lam=2.0)


def test_gaussian_and_temporal_l1_match_oracle():
    _case("Gaussian rate + temporal L1 on residual-like attributes, mode 1")
    res = synth.frame_residuals(4000, 1, 21, channels=11, sd_log_scale=0.02)[0]  # [11][n]
    _check(np.ascontiguousarray(res[7:11]), 1, 1, [1500, 4000], [0.5, 1.0], lam=1e-2, reg=1e-3)


def test_edge_cases_constant_empty_outlier():
    _case("KDE and Gaussian: constant channel, empty layer, far outlier, tiny layers")
    rng = np.random.default_rng(5)
    a = np.zeros((3, 600), np.float32)
    a[0] = 0.25                                   # all symbols equal: the bandwidth floor
    a[1] = rng.normal(0, 0.1, 600)
    a[1, 17] = 40.0                               # one far outlier: the grid spacing widens
    a[2] = rng.normal(1.0, 0.5, 600)
    lv, lw = [1, 1, 300, 600], [0.5, 0.5, 0.5, 1.0]   # a one-symbol layer and an empty one
    for kind in (0, 1):
        _check(a, kind, 1, lv, lw, reg=0.01 if kind else 0.0)


def test_results_do_not_depend_on_scheduling():
    _case("KDE rate: two runs are bit-identical")
    a = _attrs(20000, 8)
    r1 = _run(a, 0, 1, [5000, 20000], [0.5, 1.0])
    r2 = _run(a, 0, 1, [5000, 20000], [0.5, 1.0])
    for x, y in zip(r1, r2):
        assert np.array_equal(np.asarray(x), np.asarray(y))


def test_fullsize_1M_x_56_sampled_segments():
    """The benchmark's workload: 1M Gaussians x 56 attributes, six layers, training mode. The
    oracle recomputes a sample of (layer, attribute) segments: each segment's density and bits
    depend only on its own symbols."""
    _case("KDE rate full size: 1M x 56, six layers, mode 1, sampled segments")
    n = 1_000_000
    p = synth.cube_scene(n, 5, 3)
    from oracle.bitstream import significance_order
    p = synth.reorder(p, significance_order(p))
    attrs = np.ascontiguousarray(p[3:59])
    lv = synth.nested_levels(n)
    lw = synth.paper_level_weights(6)
    bits, loss, sym, grad = _run(attrs, 0, 1, lv, lw, lam=1e-7, seed=3, offset=0)
    y = E.symbols(attrs, Q, 1, 3, 0)
    bounds = [0] + list(lv)
    rng = np.random.default_rng(1)
    for l, a in [(0, 0), (5, 55), (2, 7)] + [(int(rng.integers(6)), int(rng.integers(56))) for _ in range(5)]:
        s0, s1 = bounds[l], bounds[l + 1]
        rb, rd = E.kde_bits(y[a, s0:s1], Q)
        floor_bits = -np.log2(E.P_FLOOR)
        ok = np.abs(rb - floor_bits) >= 2e-4 * floor_bits
        assert np.all(np.abs(sym[a, s0:s1] - rb)[ok] <= 1e-4 + 1e-5 * rb[ok]), (l, a)
        w = 1e-7 * lw[l] / (s1 - s0)
        r = w * rd
        assert np.abs(grad[a, s0:s1] - r)[ok].max() <= 1e-3 * np.abs(r).max(), (l, a)
    print(f"KDE bits {bits.sum():.4g}, loss {loss:.4g}", flush=True)
