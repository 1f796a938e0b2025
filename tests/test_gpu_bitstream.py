"""GPU parity of the significance order and the quantise-to-2D-maps step (gs_significance_order,
gs_encode_maps, gs_decode_maps through the C ABI) against the oracle.

The order is an integer result decided by FP32 comparisons of Psi: the GPU's order must be a
permutation that is non-increasing in the oracle's FP64 Psi up to the FP32 evaluation band
(16 ulp), equal to the oracle's order wherever no two neighbours are that close, with equal keys
ordered by index. Quantisation codes, map layout and ranges are integer (or exact) results and
must match bit for bit, given the same order; decoded values within 2 ulp of the FP64 decode.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import bitstream as BS

pytestmark = pytest.mark.gpu
BAND = 16 * 2.0 ** -24


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return torch.device("cuda:0")


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


def _check_order(p_host, order, psi_gpu):
    n = p_host.shape[1]
    psi64 = BS.significance(p_host)
    assert np.array_equal(np.sort(order), np.arange(n))
    assert np.all(np.abs(psi_gpu - psi64) <= BAND * psi64)
    seq = psi64[order]
    assert np.all(seq[1:] <= seq[:-1] * (1 + BAND))
    ps = psi_gpu[order]
    eq = ps[1:] == ps[:-1]
    assert np.all(order[1:][eq] > order[:-1][eq])  # equal FP32 keys by index
    ref = BS.significance_order(p_host)
    srt = psi64[ref]
    gaps = (srt[:-1] - srt[1:]) / srt[:-1]
    close = np.count_nonzero(gaps <= BAND)
    if close == 0:
        assert np.array_equal(order, ref)
    else:  # the differences can only be among near-ties
        diff = np.nonzero(order != ref)[0]
        for r in diff:
            assert abs(psi64[order[r]] - psi64[ref[r]]) <= 2 * BAND * psi64[ref[r]]
    return close


@pytest.mark.parametrize("n,seed", [(1, 1), (777, 2), (5000, 3)])
def test_significance_order_matches_oracle(n, seed):
    _case(f"significance order n={n}")
    from paper_2509_17513_amd.bitstream import significance_order
    dev = _dev()
    p = synth.cube_scene(n, seed, 1)
    order, psi = significance_order(torch.from_numpy(p).to(dev), with_psi=True)
    torch.cuda.synchronize()
    close = _check_order(p, order.cpu().numpy().astype(np.int64), psi.cpu().numpy().astype(np.float64))
    print(f"near-ties within the FP32 band: {close}")


def test_significance_ties_go_by_index():
    _case("significance order with duplicated Gaussians")
    from paper_2509_17513_amd.bitstream import significance_order
    p = synth.cube_scene(400, 5, 0)
    p = np.ascontiguousarray(np.concatenate([p, p[:, ::-1], p], axis=1))
    order = significance_order(torch.from_numpy(p).to(_dev())).cpu().numpy().astype(np.int64)
    assert np.array_equal(order, BS.significance_order(p))


def _gpu_encode(p, order, lv):
    from paper_2509_17513_amd.bitstream import encode_maps, planes
    dev = _dev()
    lo, ranges, maps, seq = encode_maps(torch.from_numpy(p).to(dev), torch.from_numpy(order.astype(np.int32)).to(dev),
                                        lv, with_seq=True)
    torch.cuda.synchronize()
    pl = [[t.cpu().numpy().astype(np.int64) for t in layer] for layer in planes(lo, maps)]
    return lo, ranges, maps, seq.cpu().numpy().astype(np.int64), pl


def _check_encode(p, lv):
    order = BS.significance_order(p)
    lo, ranges, maps, seq, pl = _gpu_encode(p, order, lv)
    r_ref, m_ref, s_ref = BS.encode(p, order, lv)
    assert np.array_equal(ranges.cpu().numpy(), r_ref)
    for l in range(len(lv)):
        assert pl[l][0].shape == m_ref[l].shape[1:], l
        for c in range(p.shape[0]):
            assert np.array_equal(pl[l][c], m_ref[l][c]), (l, c)
    assert np.array_equal(seq, np.concatenate(s_ref))
    from paper_2509_17513_amd.bitstream import decode_maps
    dec = decode_maps(lo, maps, ranges).cpu().numpy().astype(np.float64)
    ref = BS.decode(r_ref, m_ref, lv)
    scale = np.abs(r_ref).max(axis=2).max(axis=0)  # per channel, the largest |min|, |max|
    err = np.abs(dec - ref) / np.maximum(scale[:, None], 1e-30)
    assert err.max() <= 2 * 2.0 ** -23, err.max()
    return dec, seq


def test_encode_decode_match_oracle_with_ragged_and_empty_layers():
    _case("encode / decode 3000 Gaussians, SH 1, layers 300 / 300 (empty) / 900 / 3000")
    p = synth.cube_scene(3000, 7, 1)
    _check_encode(p, [300, 300, 900, 3000])


@pytest.mark.parametrize("n", [1, 255, 257])
def test_encode_tiny_layers(n):
    _case(f"encode / decode n={n}, one layer")
    p = synth.cube_scene(n, 11 + n, 0)
    _check_encode(p, [n])


def test_fullsize_300k_six_layers():
    _case("significance order + encode / decode, 300k Gaussians SH 3, six layers")
    from paper_2509_17513_amd.bitstream import significance_order
    w = synth.config_batched()
    p = w.params
    order = significance_order(torch.from_numpy(p).to(_dev()), with_psi=True)
    torch.cuda.synchronize()
    close = _check_order(p, order[0].cpu().numpy().astype(np.int64), order[1].cpu().numpy().astype(np.float64))
    print(f"near-ties within the FP32 band: {close}", flush=True)
    dec, seq = _check_encode(p, list(w.level_counts))
    # decoded values within half a quantisation step (plus FP32 rounding) of the originals
    lo = [0] + list(w.level_counts)
    r_ref, _, _ = BS.encode(p, BS.significance_order(p), list(w.level_counts))
    for l in range(6):
        sl = slice(lo[l], lo[l + 1])
        step = (r_ref[l, :, 1].astype(np.float64) - r_ref[l, :, 0]) / np.array(
            [2 ** BS.channel_bits(c) - 1 for c in range(p.shape[0])])
        err = np.abs(dec[:, sl] - p[:, seq[sl]])
        bits = np.array([BS.channel_bits(c) for c in range(p.shape[0])])
        assert np.all(err <= ((0.5 + 2.0 ** bits * 2.0 ** -22) * step)[:, None] + 1e-6)
