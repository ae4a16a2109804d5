"""Pins of the FP64 network reference (CPU only).

The network is not part of the paper; its reference is pinned to brute-force
loop definitions of each layer, to adjoint identities of the resampling
steps, and to central finite differences of the whole loss."""

import numpy as np
import pytest

from oracle import netref


def conv_loops(x, W, b):
    C, H, Wd = x.shape
    out = np.zeros((W.shape[0], H, Wd))
    for co in range(W.shape[0]):
        for i in range(H):
            for j in range(Wd):
                s = b[co]
                for ci in range(C):
                    for dy in range(3):
                        for dx in range(3):
                            ii, jj = i + dy - 1, j + dx - 1
                            if 0 <= ii < H and 0 <= jj < Wd:
                                s += W[co, ci, dy, dx] * x[ci, ii, jj]
                out[co, i, j] = s
    return out


def test_conv_matches_loops():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 5, 7))
    W = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    np.testing.assert_allclose(netref.conv(x, W, b), conv_loops(x, W, b), rtol=0, atol=1e-12)


def test_conv_orientation():
    # one-hot kernel at tap (dy, dx) shifts the image by (dy - 1, dx - 1)
    x = np.arange(20.0).reshape(1, 4, 5)
    W = np.zeros((1, 1, 3, 3))
    W[0, 0, 2, 0] = 1.0  # out[i][j] = x[i + 1][j - 1]
    out = netref.conv(x, W, np.zeros(1))[0]
    assert out[0, 1] == x[0, 1, 0] and out[2, 4] == x[0, 3, 3]
    assert out[3, 2] == 0.0 and out[1, 0] == 0.0


def test_conv_backward_matches_loops():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 4, 5))
    W = rng.standard_normal((3, 2, 3, 3))
    d = rng.standard_normal((3, 4, 5))
    dx, dW, db = netref.conv_backward(x, W, d)
    # the output is linear in x, W and b: gradients are the loop sums
    for idx in np.ndindex(x.shape):
        e = np.zeros_like(x)
        e[idx] = 1.0
        assert abs(dx[idx] - (d * conv_loops(e, W, np.zeros(3))).sum()) < 1e-12
    for idx in np.ndindex(W.shape):
        e = np.zeros_like(W)
        e[idx] = 1.0
        assert abs(dW[idx] - (d * conv_loops(x, e, np.zeros(3))).sum()) < 1e-12
    np.testing.assert_allclose(db, d.sum(axis=(1, 2)), atol=1e-12)


def test_resampling_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 6, 8))
    y = rng.standard_normal((2, 3, 4))
    assert abs((netref.pool(x) * y).sum() - (x * netref.pool_backward(y)).sum()) < 1e-12
    assert abs((netref.up(y) * x).sum() - (y * netref.up_backward(x)).sum()) < 1e-12
    assert netref.pool(x)[1, 2, 3] == pytest.approx(x[1, 4:6, 6:8].mean())
    assert netref.up(y)[0, 5, 7] == y[0, 2, 3]


def test_scale_equivariance_and_zero():
    p = netref.init_params(4)
    r = np.random.default_rng(5).standard_normal((2, 8, 12))
    z = netref.forward(p, r)
    np.testing.assert_allclose(netref.forward(p, 7.5 * r), 7.5 * z, rtol=1e-12, atol=1e-12)
    # zero residual: the input scale is 1, the image is the biases' response
    Ws, bs = netref.unflatten(p)
    Wz = [np.zeros_like(w) for w in Ws]
    z0 = netref.forward(netref.flatten(Wz, bs), np.zeros((1, 4, 4)))
    np.testing.assert_allclose(z0, bs[8][0], atol=0)


def test_layer_count_and_params():
    assert netref.LAYERS[6] == (96, 32) and netref.LAYERS[7] == (48, 16)
    n = sum(ci * co * 9 + co for ci, co in netref.LAYERS)
    assert netref.init_params(0).size == n
    Ws, bs = netref.unflatten(np.arange(n, dtype=np.float64))
    assert Ws[0][0, 0, 0, 0] == 0 and Ws[0][1, 0, 0, 0] == 9 and bs[0][0] == sum(ci * co * 9 for ci, co in netref.LAYERS)


def test_loss_closed_form_for_zero_net():
    p = np.zeros(netref.init_params(0).size)
    rng = np.random.default_rng(6)
    r = rng.standard_normal((2, 4, 8))
    e = rng.standard_normal((2, 4, 8))
    s = np.sqrt((r * r).mean(axis=(1, 2)))
    expect = ((e / s[:, None, None]) ** 2).mean()
    L, g = netref.gradients(p, r, e)
    assert L == pytest.approx(expect, rel=1e-14)
    assert netref.loss(p, r, e) == pytest.approx(expect, rel=1e-14)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(7)
    p = netref.init_params(8)
    r = rng.standard_normal((2, 8, 8))
    e = rng.standard_normal((2, 8, 8))
    L, g = netref.gradients(p, r, e)
    assert L == pytest.approx(netref.loss(p, r, e), rel=1e-13)
    # every layer's weights and biases, including both skip paths
    Ws, bs = netref.unflatten(np.arange(p.size, dtype=np.float64))
    idx = []
    for l in range(9):
        flat_w = Ws[l].ravel().astype(int)
        idx += list(rng.choice(flat_w, 4, replace=False)) + [int(bs[l][0])]
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (netref.loss(pp, r, e) - netref.loss(pm, r, e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])
