"""Pins of the oracle's learned-predictor network (oracle/cnn.py).

Independent checks: SciPy's correlate for the convolution, central finite
differences of the float64 loss for the backward pass, adjoint identities of
pooling and upsampling, PyTorch's bfloat16 conversion for the rounding, and
the closed form of Adam's first step.
"""

import numpy as np
import pytest
import torch
from scipy import signal

from oracle import cnn


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 9, 11, 3))
    W = rng.standard_normal((9, 4, 3))
    b = rng.standard_normal(4)
    y = cnn.conv(x, W, b, 3)
    for bi in range(2):
        for co in range(4):
            ref = np.full((9, 11), b[co])
            for ci in range(3):
                k = W[:, co, ci].reshape(3, 3)
                ref += signal.correlate(x[bi, :, :, ci], k, mode="same")
            np.testing.assert_allclose(y[bi, :, :, co], ref, atol=1e-12)


def test_conv_backward_fd():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 5, 6, 2))
    W = rng.standard_normal((9, 3, 2))
    b = rng.standard_normal(3)
    dy = rng.standard_normal((1, 5, 6, 3))
    dx, dW, db = cnn.conv_backward(x, W, 3, dy)
    f = lambda x_, W_, b_: float(np.sum(cnn.conv(x_, W_, b_, 3) * dy))
    eps = 1e-6
    for idx in [(0, 2, 3, 1), (0, 0, 0, 0), (0, 4, 5, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        assert dx[idx] == pytest.approx((f(xp, W, b) - f(xm, W, b)) / 2 / eps,
                                        rel=1e-6)
    for idx in [(4, 1, 0), (0, 2, 1), (8, 0, 1)]:
        Wp, Wm = W.copy(), W.copy()
        Wp[idx] += eps
        Wm[idx] -= eps
        assert dW[idx] == pytest.approx((f(x, Wp, b) - f(x, Wm, b)) / 2 / eps,
                                        rel=1e-6)
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2)))


def test_pool_up_adjoint():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 8, 6, 3))
    y = rng.standard_normal((2, 4, 3, 3))
    assert np.sum(cnn.pool(x) * y) == pytest.approx(
        np.sum(x * cnn.pool_backward(y)), rel=1e-12)
    assert np.sum(cnn.up(y) * x) == pytest.approx(
        np.sum(y * cnn.up_backward(x)), rel=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(
        -3, 3, 1000), [1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -0.0]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).float()
    np.testing.assert_array_equal(cnn.to_bf16(x), ref.numpy().astype(
        np.float64))


def test_network_gradient_fd_float64():
    rng = np.random.default_rng(4)
    params = cnn.init_params(5).astype(np.float64)
    x = rng.standard_normal((1, 16, 16, 7))
    tgt = rng.standard_normal((1, 16, 16, 2)) * 0.1
    loss, grad = cnn.loss_and_grad(params, x, tgt, bf16=False)
    assert grad.shape == (cnn.param_count(),)
    eps = 1e-6
    picks = rng.choice(params.size, 25, replace=False)
    for i in picks:
        pp, pm = params.copy(), params.copy()
        pp[i] += eps
        pm[i] -= eps
        lp = cnn.loss_and_grad(pp, x, tgt, bf16=False)[0]
        lm = cnn.loss_and_grad(pm, x, tgt, bf16=False)[0]
        fd = (lp - lm) / (2 * eps)
        assert grad[i] == pytest.approx(fd, rel=1e-4, abs=1e-9)
    out, _ = cnn.forward(params, x, bf16=False)
    assert loss == pytest.approx(float(np.mean((out - tgt) ** 2)), rel=1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(6)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    p1, m, v = cnn.adam(p, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> step = lr sign(g)
    np.testing.assert_allclose(p - p1, 1e-3 * np.sign(g), rtol=1e-6)


def test_layer_table():
    # encoder 32/64/128/128, decoder with skip concatenations, 1x1 head
    chans = {n: (ci, co) for n, ci, co, k in cnn.LAYERS}
    assert chans["d3a"][0] == chans["e3b"][1] + chans["e4b"][1]
    assert chans["d2a"][0] == chans["e2b"][1] + chans["d3b"][1]
    assert chans["d1a"][0] == chans["e1b"][1] + chans["d2b"][1]
    assert chans["head"] == (32, 2)
    assert cnn.param_count() == cnn.init_params(0).size


# ------------------------------------------------------------------- 3-D


def test_conv3d_matches_scipy_correlate():
    rng = np.random.default_rng(10)
    x = rng.standard_normal((2, 5, 7, 6, 3))
    W = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(2)
    y = cnn.conv(x, W, b, 3)
    for bi in range(2):
        for co in range(2):
            ref = np.full((5, 7, 6), b[co])
            for ci in range(3):
                k = W[:, co, ci].reshape(3, 3, 3)   # tap = 9 dz + 3 dy + dx
                ref += signal.correlate(x[bi, ..., ci], k, mode="same")
            np.testing.assert_allclose(y[bi, ..., co], ref, atol=1e-12)


def test_conv3d_backward_fd():
    rng = np.random.default_rng(11)
    x = rng.standard_normal((1, 4, 5, 3, 2))
    W = rng.standard_normal((27, 2, 2))
    b = rng.standard_normal(2)
    dy = rng.standard_normal((1, 4, 5, 3, 2))
    dx, dW, db = cnn.conv_backward(x, W, 3, dy)
    f = lambda x_, W_: float(np.sum(cnn.conv(x_, W_, b, 3) * dy))
    eps = 1e-6
    for idx in [(0, 0, 0, 0, 1), (0, 3, 4, 2, 0), (0, 2, 1, 1, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        assert dx[idx] == pytest.approx((f(xp, W) - f(xm, W)) / 2 / eps,
                                        rel=1e-6)
    for idx in [(0, 1, 0), (13, 0, 1), (26, 1, 1), (9, 0, 0)]:
        Wp, Wm = W.copy(), W.copy()
        Wp[idx] += eps
        Wm[idx] -= eps
        assert dW[idx] == pytest.approx((f(x, Wp) - f(x, Wm)) / 2 / eps,
                                        rel=1e-6)
    np.testing.assert_allclose(db, dy.sum(axis=(0, 1, 2, 3)))


def test_pool3d_up3d_adjoint_and_values():
    rng = np.random.default_rng(12)
    x = rng.standard_normal((1, 4, 6, 8, 2))
    y = rng.standard_normal((1, 2, 3, 4, 2))
    assert np.sum(cnn.pool(x) * y) == pytest.approx(
        np.sum(x * cnn.pool_backward(y)), rel=1e-12)
    assert np.sum(cnn.up(y) * x) == pytest.approx(
        np.sum(y * cnn.up_backward(x)), rel=1e-12)
    # brute force: mean of the 2 x 2 x 2 block
    assert cnn.pool(x)[0, 1, 2, 3, 1] == pytest.approx(
        x[0, 2:4, 4:6, 6:8, 1].mean(), rel=1e-14)
    assert cnn.up(y)[0, 3, 5, 7, 0] == y[0, 1, 2, 3, 0]


def test_network3d_gradient_fd_float64():
    rng = np.random.default_rng(13)
    params = cnn.init_params(7, dim=3).astype(np.float64)
    x = rng.standard_normal((1, 8, 8, 8, 9))
    tgt = rng.standard_normal((1, 8, 8, 8, 3)) * 0.1
    loss, grad = cnn.loss_and_grad(params, x, tgt, bf16=False)
    assert grad.shape == (cnn.param_count(3),)
    eps = 1e-6
    # a weight and a bias of every layer, sampled
    offs, o = [], 0
    for name, ci, co, k in cnn.layers(3):
        nw = k ** 3 * co * ci
        offs += [o + int(rng.integers(nw)), o + nw + int(rng.integers(co))]
        o += nw + co
    for i in offs[::2]:
        pp, pm = params.copy(), params.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (cnn.loss_and_grad(pp, x, tgt, bf16=False)[0] -
              cnn.loss_and_grad(pm, x, tgt, bf16=False)[0]) / (2 * eps)
        assert grad[i] == pytest.approx(fd, rel=1e-4, abs=1e-9)
    out, _ = cnn.forward(params, x, bf16=False)
    assert out.shape == (1, 8, 8, 8, 3)
    assert loss == pytest.approx(float(np.mean((out - tgt) ** 2)), rel=1e-12)


def test_layer_table_3d():
    lay = {n: (ci, co, k) for n, ci, co, k in cnn.layers(3)}
    assert lay["e1a"][0] == 9            # 3 frames + 2 x 3 components
    assert lay["head"][:2] == (32, 3)
    n3 = cnn.param_count(3)
    assert n3 == cnn.init_params(0, dim=3).size
    # every 3x3 layer has 18 more taps than in 2-D; e1a has 2 more input
    # channels (9 taps each in 2-D) and the head one more output channel
    diff = sum(18 * ci * co for n, (ci, co, k) in lay.items() if k == 3)
    diff += 9 * 2 * 32 + (32 + 1)
    assert n3 - cnn.param_count(2) == diff
