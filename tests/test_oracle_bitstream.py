"""Pins of the significance-order and quantise-to-2D-maps oracle: the metric's closed form and a
brute-force sort, bit interleaving against a per-bit loop, the map layout as a bijection made of
whole 16 x 16 blocks, the quantiser's end points and round-trip error, and encode/decode."""
import numpy as np
import pytest

from oracle import bitstream as BS


def _params(n, seed, C=14):
    rng = np.random.default_rng(seed)
    p = np.zeros((C, n), np.float32)
    p[0:3] = rng.uniform(-1, 1, (3, n))
    p[3:6] = rng.normal(-3, 0.5, (3, n))
    p[6:10] = rng.normal(0, 1, (4, n))
    p[10] = rng.normal(0, 1.5, n)
    p[11:] = rng.normal(0, 0.3, (C - 11, n))
    return p


def test_significance_closed_form_and_order():
    p = np.zeros((14, 3), np.float32)
    p[3:6, 0] = [np.log(0.1), np.log(0.2), np.log(0.3)]
    p[10, 0] = 0.0
    p[3:6, 1] = -10.0
    p[10, 1] = 2.0
    p[3:6, 2] = [np.log(0.1), np.log(0.3), np.log(0.2)]  # same volume as Gaussian 0
    psi = BS.significance(p, 1e5)
    # the log-scales are stored in FP32, so the volume matches to FP32 rounding
    assert abs(psi[0] - (0.5 + 1e5 * 4 / 3 * np.pi * 0.1 * 0.2 * 0.3)) < 1e-6 * psi[0]
    assert abs(psi[1] - (1 / (1 + np.exp(-2.0)) + 1e5 * 4 / 3 * np.pi * np.exp(-30.0))) < 1e-12
    # ties by lower index; Gaussian 1 is last
    assert list(BS.significance_order(p)) in ([0, 2, 1], [2, 0, 1])
    q = _params(500, 1)
    psi = BS.significance(q)
    ref = sorted(range(500), key=lambda i: (-psi[i], i))
    assert list(BS.significance_order(q)) == ref


def test_morton_against_bit_loop():
    rng = np.random.default_rng(2)
    x, y, z = rng.integers(0, 1024, 200), rng.integers(0, 1024, 200), rng.integers(0, 512, 200)
    got = BS.morton3(x, y, z)
    for i in range(200):
        ref = 0
        for k in range(30):
            axis, bit = k % 3, k // 3
            src = (int(x[i]), int(y[i]), int(z[i]))[axis]
            ref |= ((src >> bit) & 1) << k
        assert got[i] == ref


@pytest.mark.parametrize("m,w,h", [(1, 16, 16), (256, 16, 16), (257, 32, 16), (1000, 32, 32),
                                   (300_000, 560, 544), (25_000, 160, 160)])
def test_map_sizes(m, w, h):
    assert BS.map_size(m) == (w, h)


@pytest.mark.parametrize("w,h", [(16, 16), (48, 32), (160, 160)])
def test_layout_is_a_bijection_of_whole_blocks(w, h):
    x, y = BS.block_pixel(np.arange(w * h), w)
    assert x.min() == 0 and y.min() == 0 and x.max() == w - 1 and y.max() == h - 1
    assert len(set(zip(x.tolist(), y.tolist()))) == w * h
    bx, by = x // 16, y // 16
    for b in range(w * h // 256):
        sl = slice(256 * b, 256 * (b + 1))
        assert len(set(zip(bx[sl].tolist(), by[sl].tolist()))) == 1  # one block per 256 positions
    # consecutive blocks touch (snake), and the 2D Morton curve starts at the block corner
    blocks = list(zip(bx[::256].tolist(), by[::256].tolist()))
    for a, b in zip(blocks, blocks[1:]):
        assert abs(a[0] - b[0]) + abs(a[1] - b[1]) == 1
    assert (x[0], y[0], x[1], y[1], x[2], y[2], x[3], y[3]) == (0, 0, 1, 0, 0, 1, 1, 1)


def test_quantiser_end_points_and_round_trip():
    rng = np.random.default_rng(3)
    for bits in (8, 16):
        v = rng.uniform(-2.5, 4.0, 5000).astype(np.float32)
        mn, mx = v.min(), v.max()
        code = BS.quantise(v, mn, mx, bits)
        assert code.min() == 0 and code.max() == 2 ** bits - 1
        assert code[np.argmin(v)] == 0 and code[np.argmax(v)] == 2 ** bits - 1
        step = (float(mx) - float(mn)) / (2 ** bits - 1)
        err = np.abs(BS.dequantise(code, mn, mx, bits) - v)
        # half a step, plus the FP32 rounding of (v - min) * scale (a few ulp of 2^b - 1 codes)
        assert err.max() <= (0.5 + 2.0 ** bits * 2.0 ** -22) * step
    assert (BS.quantise(np.full(7, 0.3, np.float32), 0.3, 0.3, 8) == 0).all()


def test_encode_decode_round_trip():
    p = _params(3000, 4)
    lv = [300, 900, 3000]
    order = BS.significance_order(p)
    ranges, maps, seqs = BS.encode(p, order, lv)
    assert [m.shape for m in maps] == [(14, 16, 32), (14, 32, 32), (14, 48, 48)]
    # every layer's sequence is a permutation of its ranks' Gaussians
    bounds = [0] + lv
    for l in range(3):
        assert sorted(seqs[l].tolist()) == sorted(order[bounds[l]:bounds[l + 1]].tolist())
    dec = BS.decode(ranges, maps, lv)
    src = np.concatenate(seqs)
    for c in range(14):
        bits = BS.channel_bits(c)
        for l in range(3):
            step = (float(ranges[l, c, 1]) - float(ranges[l, c, 0])) / (2 ** bits - 1)
            sl = slice(bounds[l], bounds[l + 1])
            assert np.abs(dec[c, sl] - p[c, src[sl]]).max() <= (0.5 + 2.0 ** bits * 2.0 ** -22) * step + 1e-7
    # the Morton order makes neighbours in the sequence close in space: mean step << random
    pos = p[0:3, seqs[2]]
    seq_step = np.linalg.norm(np.diff(pos, axis=1), axis=0).mean()
    rnd_step = np.linalg.norm(np.diff(p[0:3, np.random.default_rng(5).permutation(seqs[2])], axis=1), axis=0).mean()
    assert seq_step < 0.3 * rnd_step
