"""Pins for the learned-density network oracle: conv against an explicit
per-voxel sum, backward pass against central finite differences, and the
inference post-processing invariants."""
import numpy as np
import pytest

from oracle import convnet as cn


def _small_params(seed=3, scale=0.5):
    rng = np.random.default_rng(seed)
    return [(scale * rng.standard_normal((co, ci, 3, 3, 3)), 0.1 * rng.standard_normal(co))
            for ci, co in [(1, 3), (3, 3), (3, 2), (2, 1)]]


def test_conv_matches_explicit_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4, 5, 3))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    out = cn.conv(x, W, b)
    S = x.shape[1:]
    for co in range(3):
        for r in [(0, 0, 0), (3, 4, 2), (1, 2, 1)]:
            v = b[co]
            for ci in range(2):
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            v += W[co, ci, dz + 1, dy + 1, dx + 1] * x[ci, (r[0] + dz) % S[0], (r[1] + dy) % S[1],
                                                                      (r[2] + dx) % S[2]]
            assert abs(out[co][r] - v) < 1e-12


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    params = _small_params()
    x = rng.standard_normal((1, 5, 4, 6))
    t = rng.standard_normal((5, 4, 6))
    L, grads = cn.loss_and_grads(params, x, t)
    h = 1e-6
    for l in range(4):
        W, b = params[l]
        for idx in [(0, 0, 1, 1, 1), (W.shape[0] - 1, W.shape[1] - 1, 0, 2, 1)]:
            Wp = W.copy()
            Wp[idx] += h
            Wm = W.copy()
            Wm[idx] -= h
            Lp = cn.loss_and_grads([p if i != l else (Wp, b) for i, p in enumerate(params)], x, t)[0]
            Lm = cn.loss_and_grads([p if i != l else (Wm, b) for i, p in enumerate(params)], x, t)[0]
            fd = (Lp - Lm) / (2 * h)
            assert abs(fd - grads[l][0][idx]) < 1e-6 * max(1.0, abs(fd))
        bp = b.copy()
        bp[0] += h
        bm = b.copy()
        bm[0] -= h
        Lp = cn.loss_and_grads([p if i != l else (W, bp) for i, p in enumerate(params)], x, t)[0]
        Lm = cn.loss_and_grads([p if i != l else (W, bm) for i, p in enumerate(params)], x, t)[0]
        assert abs((Lp - Lm) / (2 * h) - grads[l][1][0]) < 1e-6


def test_input_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    W = rng.standard_normal((2, 3, 3, 3, 3))
    x = rng.standard_normal((3, 4, 5, 4))
    dout = rng.standard_normal((2, 4, 5, 4))
    dx, dW, db = cn.conv_backward(x, W, dout)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (2, 3, 4, 1), (1, 1, 2, 3)]:
        xp = x.copy()
        xp[idx] += h
        xm = x.copy()
        xm[idx] -= h
        fd = (np.sum(dout * cn.conv(xp, W, np.zeros(2))) - np.sum(dout * cn.conv(xm, W, np.zeros(2)))) / (2 * h)
        assert abs(fd - dx[idx]) < 1e-6


def test_prediction_is_normalized_and_nonnegative():
    params = cn.init_params(501)
    assert sum(W.size + b.size for W, b in params) == 14737
    rng = np.random.default_rng(4)
    n0 = rng.gamma(2.0, 0.01, (8, 8, 8))
    n = cn.predict_density(params, n0, 32.0, 1000.0)
    assert np.all(n >= 0)
    assert abs(1000.0 / n.size * n.sum() - 32.0) < 1e-10


def test_adam_moves_against_gradient():
    params = _small_params()
    grads = [(np.ones_like(W), np.ones_like(b)) for W, b in params]
    opt = cn.Adam(params, lr=1e-2)
    new = opt.step(params, grads)
    # the first Adam step moves every parameter by -lr * sign(g)
    for (W0, b0), (W1, b1) in zip(params, new):
        assert np.allclose(W1 - W0, -1e-2, atol=1e-9)
