"""GPU parity of the rate path (HIP kernels through the C ABI) against the FP64 rate oracle:
histogram rate (exact counts), context features, the BF16-MFMA Laplace MLP forward (bits) and
backward (attribute, weight and bias gradients), and the Adam update."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import rate

pytestmark = pytest.mark.gpu
Q = 1.0 / 64


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _lib():
    from paper_2509_17513_amd import _lib
    return _lib


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _attrs(n, seed=61):
    p = synth.cube_scene(n, seed, 3)
    return np.ascontiguousarray(p[3:]), np.ascontiguousarray(p[0:3])


def _desc(n, A, mode, lv=None, lw=None, lam=1.0, seed=0, offset=0, fit=None):
    L = _lib()
    d = L.GsRateDesc()
    d.n, d.n_attr, d.step, d.mode, d.seed, d.offset = n, A, Q, mode, seed, offset
    lv = lv or [n]
    lw = lw or [1.0] * len(lv)
    d.n_levels = len(lv)
    for i, v in enumerate(lv):
        d.level_counts[i] = v
        d.level_weights[i] = lw[i]
    d.lambda_rate = lam
    d.fit_scale = 1.0 / n if fit is None else fit
    return d


@pytest.mark.parametrize("n", [1, 777, 20000])
def test_histogram_bits_exact(n):
    _case(f"histogram rate n={n}")
    L = _lib()
    dev = torch.device("cuda:0")
    attrs, _ = _attrs(n)
    A = attrs.shape[0]
    a = torch.from_numpy(attrs).to(dev)
    sz = ctypes.c_size_t()
    assert L.lib().gs_rate_histogram_workspace_size(A, ctypes.byref(sz)) == 0
    ws = torch.zeros(sz.value, dtype=torch.uint8, device=dev)
    bits = torch.zeros(A, dtype=torch.float64, device=dev)
    L.check(L.lib().gs_rate_histogram(n, A, _p(a), ctypes.c_float(Q), _p(bits), _p(ws), sz.value, _stream()),
            "gs_rate_histogram")
    torch.cuda.synchronize()
    ref = rate.hist_bits(attrs, Q)
    np.testing.assert_allclose(bits.cpu().numpy(), ref, rtol=1e-12, atol=1e-9)


def test_context_features():
    _case("context features")
    L = _lib()
    dev = torch.device("cuda:0")
    n = 5000
    _, means = _attrs(n)
    lv = [500, 1000, 2500, 5000]
    m = torch.from_numpy(means).to(dev)
    ctx = torch.zeros((n, 16), dtype=torch.int16, device=dev)
    lvc = (ctypes.c_int32 * 4)(*lv)
    L.check(L.lib().gs_rate_context(n, _p(m), ctypes.c_float(1.0), 4, lvc, _p(ctx), _stream()), "gs_rate_context")
    torch.cuda.synchronize()
    got = rate.bf16_bits_to_f64(ctx.cpu().numpy().view(np.uint16)).T  # [16][n]
    ref = rate.context(means, 1.0, rate.layer_of(n, lv))
    diff = got != ref
    # float32 sin/cos may round to the neighbouring BF16 value in rare cases
    assert diff.mean() < 1e-3
    ulp = np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)
    assert ulp[diff].max() <= 2 ** -7 + 1e-12 if diff.any() else True
    np.testing.assert_array_equal(got[15], ref[15])


def _mlp_inputs(n, A, seed):
    attrs, means = _attrs(n, seed)
    attrs = np.ascontiguousarray(attrs[:A])
    lv = [n // 4, n // 2, n]
    ctx = rate.context(means, 1.0, rate.layer_of(n, lv))  # [16][n], BF16 values
    wbits, bf = rate.init_weights(A, seed, attrs)
    return attrs, ctx, wbits, bf, lv


def _gpu_mlp(attrs, ctx, wbits, bf, lv, lw, mode, lam, seed=0, offset=0, grad=True):
    L = _lib()
    dev = torch.device("cuda:0")
    A, n = attrs.shape
    a = torch.from_numpy(attrs).to(dev)
    c = torch.from_numpy(np.ascontiguousarray(rate.f64_to_bf16_bits(ctx.T))).to(dev)
    w = torch.from_numpy(wbits.view(np.int16)).to(dev)
    b = torch.from_numpy(bf.astype(np.float32)).to(dev)
    bits = torch.zeros(A, dtype=torch.float64, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    da = torch.zeros_like(a) if mode == 1 else None
    dw = torch.zeros((A, rate.W_PER_ATTR), dtype=torch.float32, device=dev) if grad else None
    db = torch.zeros((A, rate.B_PER_ATTR), dtype=torch.float32, device=dev) if grad else None
    d = _desc(n, A, mode, lv, lw, lam, seed, offset)
    P = lambda t: None if t is None else _p(t)  # noqa: E731
    L.check(L.lib().gs_rate_model(ctypes.byref(d), _p(a), _p(c), _p(w), _p(b), _p(bits), _p(loss), None, P(da),
                                  P(dw), P(db), _stream()), "gs_rate_model")
    torch.cuda.synchronize()
    out = {"bits": bits.cpu().numpy(), "loss": float(loss.item())}
    if da is not None:
        out["d_attrs"] = da.cpu().numpy()
    if grad:
        out["d_w"] = dw.cpu().numpy()
        out["d_b"] = db.cpu().numpy()
    return out


@pytest.mark.parametrize("n", [33, 4096 + 17])
def test_mlp_eval_bits_match_oracle(n):
    _case(f"rate MLP eval n={n}")
    A = 8
    attrs, ctx, wbits, bf, lv = _mlp_inputs(n, A, 71)
    lw = [0.5, 0.25, 1.0]
    g = _gpu_mlp(attrs, ctx, wbits, bf, lv, lw, 0, 1.0, grad=False)
    ref = rate.rate_model(attrs, ctx, wbits, bf, Q, mode=0, sym_w=rate.symbol_weights(n, lv, lw, 1.0),
                          want_grad=False)
    np.testing.assert_allclose(g["bits"], ref["bits"], rtol=1e-3)
    assert abs(g["loss"] - ref["loss"]) <= 1e-3 * abs(ref["loss"])


def test_mlp_train_gradients_match_oracle():
    _case("rate MLP train mode: noise, d_attrs, d_w, d_b")
    n, A = 6000, 6
    attrs, ctx, wbits, bf, lv = _mlp_inputs(n, A, 73)
    lw = [0.5, 0.25, 1.0]
    lam = 3.0
    g = _gpu_mlp(attrs, ctx, wbits, bf, lv, lw, 1, lam, seed=99, offset=12345)
    ref = rate.rate_model(attrs, ctx, wbits, bf, Q, mode=1, seed=99, offset=12345,
                          sym_w=rate.symbol_weights(n, lv, lw, lam), fit_scale=1.0 / n, want_abs=True)
    np.testing.assert_allclose(g["bits"], ref["bits"], rtol=1e-3)
    assert abs(g["loss"] - ref["loss"]) <= 1e-3 * abs(ref["loss"])
    da, rda = g["d_attrs"], ref["d_attrs"]
    rms = np.sqrt(np.mean(rda ** 2))
    bad = np.abs(da - rda) > 2e-2 * np.abs(rda) + 1e-2 * rms
    assert bad.sum() == 0, bad.sum()
    for k in ("d_w", "d_b"):
        x, r, ra = g[k], ref[k], ref[k + "_abs"]
        for a in range(A):
            rms = np.sqrt(np.mean(r[a] ** 2)) + 1e-30
            # each term of these sums over symbols is a product of two BF16-rounded factors; where the
            # float32 and FP64 values straddle a BF16 rounding boundary the two sides round a factor to
            # neighbouring BF16 values, so a term may differ by up to 2^-7 of itself: the bar adds 2^-7
            # of the sum of the absolute terms to the relative bar
            err = np.abs(x[a] - r[a]) / (2e-2 * np.abs(r[a]) + 2e-2 * rms + 2.0 ** -7 * ra[a])
            assert np.all(err <= 1), (k, a, np.mean(err > 1), err.max())
            np.testing.assert_allclose(np.linalg.norm(x[a]), np.linalg.norm(r[a]), rtol=2e-2)


def test_rate_autotune_picks_an_agreeing_launch_shape():
    _case("rate autotuner: candidates agree, tuned launch equals the default")
    L = _lib()
    n, A = 200_000, 4
    attrs, ctx, wbits, bf, lv = _mlp_inputs(n, A, 79)
    lw = [0.5, 0.25, 1.0]
    dev = torch.device("cuda:0")
    a = torch.from_numpy(attrs).to(dev)
    c = torch.from_numpy(np.ascontiguousarray(rate.f64_to_bf16_bits(ctx.T))).to(dev)
    w = torch.from_numpy(wbits.view(np.int16)).to(dev)
    b = torch.from_numpy(bf.astype(np.float32)).to(dev)
    scratch = torch.zeros((5, A), dtype=torch.float64, device=dev)
    da = torch.zeros_like(a)
    dw = torch.zeros((A, rate.W_PER_ATTR), dtype=torch.float32, device=dev)
    db = torch.zeros((A, rate.B_PER_ATTR), dtype=torch.float32, device=dev)
    best = ctypes.c_int32()
    times = (ctypes.c_float * 5)()
    d = _desc(n, A, 1, lv, lw, 1.0, seed=5)
    L.check(L.lib().gs_rate_autotune(ctypes.byref(d), _p(a), _p(c), _p(w), _p(b), _p(scratch), _p(da), _p(dw),
                                     _p(db), _stream(), ctypes.byref(best), times), "gs_rate_autotune")
    t = list(times)
    print(f"best={best.value} times={t}")
    assert best.value in (16, 32, 64, 128, 256)
    assert all(x > 0 for x in t)  # every launch shape gives the same bits
    assert t[(16, 32, 64, 128, 256).index(best.value)] == min(t)
    sb = scratch.cpu().numpy()
    np.testing.assert_allclose(sb, np.broadcast_to(sb[0], sb.shape), rtol=1e-5)
    outs = []
    for blocks in (0, best.value):
        bits = torch.zeros(A, dtype=torch.float64, device=dev)
        gw = torch.zeros_like(dw)
        d.blocks_per_attr = blocks
        L.check(L.lib().gs_rate_model(ctypes.byref(d), _p(a), _p(c), _p(w), _p(b), _p(bits), None, None, None,
                                      _p(gw), None, _stream()), "gs_rate_model")
        torch.cuda.synchronize()
        outs.append((bits.cpu().numpy(), gw.cpu().numpy()))
    np.testing.assert_allclose(outs[1][0], outs[0][0], rtol=1e-5)
    np.testing.assert_allclose(outs[1][1], outs[0][1], rtol=1e-3, atol=1e-4 * np.abs(outs[0][1]).max())


def test_adam_step_matches_reference():
    _case("Adam")
    L = _lib()
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(5)
    n = 10007
    p0 = rng.standard_normal(n).astype(np.float32)
    g0 = rng.standard_normal(n).astype(np.float32)
    m0 = rng.standard_normal(n).astype(np.float32) * 0.1
    v0 = rng.uniform(0, 1, n).astype(np.float32)
    p, g, m, v = (torch.from_numpy(x.copy()).to(dev) for x in (p0, g0, m0, v0))
    cp = torch.zeros(n, dtype=torch.int16, device=dev)
    lr, b1, b2, eps, t = 1e-2, 0.9, 0.999, 1e-8, 7
    L.check(L.lib().gs_adam_step(n, _p(p), _p(g), _p(m), _p(v), _p(cp), ctypes.c_float(lr), ctypes.c_float(b1),
                                 ctypes.c_float(b2), ctypes.c_float(eps), t, _stream()), "gs_adam_step")
    torch.cuda.synchronize()
    mr = b1 * m0.astype(np.float64) + (1 - b1) * g0
    vr = b2 * v0.astype(np.float64) + (1 - b2) * g0.astype(np.float64) ** 2
    pr = p0 - lr * (mr / (1 - b1 ** t)) / (np.sqrt(vr / (1 - b2 ** t)) + eps)
    np.testing.assert_allclose(p.cpu().numpy(), pr, rtol=1e-5, atol=1e-6)
    assert torch.all(g == 0)
    np.testing.assert_array_equal(rate.bf16_bits_to_f64(cp.cpu().numpy().view(np.uint16)),
                                  rate.bf16_round(p.cpu().numpy().astype(np.float64)))


def test_initial_output_bias_is_the_context_free_laplace_fit():
    _case("gs_rate_init_output_bias: mean and mean absolute deviation per attribute, on the device")
    from paper_2509_17513_amd.train import RateModel
    dev = torch.device("cuda:0")
    n, A = 100_003, 7
    rng = np.random.default_rng(61)
    y = np.stack([rng.laplace(0.05 * a, 0.02 + 0.01 * a, n) for a in range(A)]).astype(np.float32)
    y[3] = 0.25  # a constant attribute: MAD 0 -> the scale floor step / 4
    rm = RateModel(A, dev, seed=3, attrs=torch.from_numpy(y).to(dev))
    torch.cuda.synchronize()
    b = rm.b.cpu().numpy()
    y64 = y.astype(np.float64)
    mean = y64.mean(axis=1)
    mad = np.abs(y64 - mean[:, None]).mean(axis=1)
    target = np.maximum(mad - Q / 16, Q / 4)
    np.testing.assert_allclose(b[:, 128], mean.astype(np.float32), rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(b[:, 129], np.log(np.expm1(target)).astype(np.float32), rtol=1e-6, atol=1e-6)
    assert np.all(b[:, :128] == 0.0)
