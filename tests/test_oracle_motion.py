"""Pins of the rigid-motion oracle (hash-grid encoding + two MLPs): level resolutions, the
spatial hash against Python integers, trilinear interpolation reproducing a linear field on the
dense levels, the identity at zero weights, clamping outside the scene box, and the backward
against central differences."""
import numpy as np

import synth
from oracle import motion as M

LO, HI = np.array([-1.0, -1.0, -1.0]), np.array([1.0, 1.0, 1.0])


def _params(seed, **kw):
    shapes = [s for out in (3, 4) for s in M.head_sizes(out)]
    return synth.motion_params(seed, M.LEVELS * M.T * M.FEATS, shapes, **kw)


def test_resolutions_and_dense_levels():
    r = M.resolutions()
    assert r[0] == 16 and r[-1] == 1024 and all(a < b for a, b in zip(r, r[1:]))
    dense = [N for N in r if (N + 1) ** 3 <= M.T]
    assert len(dense) == 3  # both indexings are exercised


def test_hash_against_python_integers():
    rng = np.random.default_rng(1)
    for _ in range(200):
        i, j, k = (int(v) for v in rng.integers(0, 1025, 3))
        ref = ((i * 1) % 2 ** 32 ^ (j * 2654435761) % 2 ** 32 ^ (k * 805459861) % 2 ** 32) % M.T
        assert M.corner_index(np.array([i]), np.array([j]), np.array([k]), 1024)[0] == ref


def test_trilinear_reproduces_linear_fields_on_dense_levels():
    rng = np.random.default_rng(2)
    table = np.zeros((M.LEVELS, M.T, M.FEATS))
    coef = rng.normal(0, 1, (M.LEVELS, 4))
    for l, N in enumerate(M.resolutions()):
        if (N + 1) ** 3 > M.T:
            continue
        i, j, k = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
        idx = M.corner_index(i.ravel(), j.ravel(), k.ravel(), N)
        table[l, idx, 0] = coef[l, 0] * i.ravel() + coef[l, 1] * j.ravel() + coef[l, 2] * k.ravel() + coef[l, 3]
    mu = rng.uniform(-1, 1, (3, 500))
    h, _ = M.encode(mu, LO, HI, table)
    p = (mu.T - LO) / (HI - LO)
    for l, N in enumerate(M.resolutions()):
        if (N + 1) ** 3 > M.T:
            continue
        x = p * N
        exp = coef[l, 0] * x[:, 0] + coef[l, 1] * x[:, 1] + coef[l, 2] * x[:, 2] + coef[l, 3]
        np.testing.assert_allclose(h[:, 2 * l], exp, rtol=1e-12, atol=1e-12)


def test_identity_at_zero_weights_and_clamping():
    table, w = _params(3)
    out = M.forward(np.random.default_rng(3).uniform(-1, 1, (3, 50)), LO, HI, table, np.zeros_like(w))
    assert np.all(out[0:3] == 0) and np.all(out[3] == 1) and np.all(out[4:7] == 0)
    # outside the box: the same features as the box's face
    mu = np.array([[0.3, 0.3], [5.0, 1.0], [-0.2, -0.2]])
    h, _ = M.encode(mu, LO, HI, table)
    np.testing.assert_allclose(h[0], h[1], rtol=0, atol=0)


def test_backward_against_central_differences():
    table, w = _params(4, table_scale=0.5)
    rng = np.random.default_rng(5)
    mu = rng.uniform(-1, 1, (3, 40))
    d_out = rng.normal(0, 1, (7, 40))
    dt, dw = M.backward(mu, LO, HI, table, w, d_out)

    def loss(tb, ww):
        return float((M.forward(mu, LO, HI, tb, ww) * d_out).sum())

    e = 1e-6
    for k in rng.choice(np.nonzero(dw)[0], 25, replace=False):
        wp, wm = w.astype(np.float64), w.astype(np.float64)
        wp[k] += e
        wm[k] -= e
        fd = (loss(table, wp) - loss(table, wm)) / (2 * e)
        assert abs(fd - dw[k]) <= 1e-5 * abs(fd) + 1e-8, ("w", k, fd, dw[k])
    for k in rng.choice(np.nonzero(dt)[0], 25, replace=False):
        tp, tm = table.astype(np.float64), table.astype(np.float64)
        tp[k] += e
        tm[k] -= e
        fd = (loss(tp, w) - loss(tm, w)) / (2 * e)
        assert abs(fd - dt[k]) <= 1e-5 * abs(fd) + 1e-8, ("t", k, fd, dt[k])
    assert M.n_weights() == dw.size == w.size
