"""Pins of the float64 surrogate reference (oracle/nn.py) against things other than itself:
numpy's correlation for the conv orientation and padding, adjoint identities for the two
backward convolutions, central finite differences for the whole gradient, closed forms for
the pooling/MLP head and for Adam's first steps, bit-level float32 rounding for bfloat16, and a
hand-computed feature table. CPU only."""
import numpy as np
import pytest

from oracle import nn


def test_bf16_round_matches_float32_bit_rounding():
    rng = np.random.default_rng(0)
    x32 = (rng.standard_normal(20000) * np.exp(rng.uniform(-10, 10, 20000))).astype(np.float32)
    bits = x32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32).view(np.float32)
    assert np.array_equal(nn.bf16_round(x32.astype(np.float64)), rounded.astype(np.float64))
    # ties go to the even significand
    assert nn.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert nn.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert nn.bf16_round(-(1.0 + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)


def test_single_channel_conv_is_numpy_correlate_same():
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 13):
        x = rng.standard_normal(n)
        w = rng.standard_normal(5)
        got = nn.conv(x[:, None], w[:, None, None])[:, 0]
        # full correlation at lags -2 .. n-3 (numpy's "same" when n >= 5)
        want = np.correlate(x, w, mode="full")[2:2 + n]
        assert np.allclose(got, want, atol=1e-12, rtol=0)
        if n >= 5:
            assert np.allclose(got, np.correlate(x, w, mode="same"), atol=1e-12, rtol=0)


def test_backward_convolutions_are_the_adjoints_of_conv():
    rng = np.random.default_rng(2)
    n, ci, co = 11, 6, 7
    H = rng.standard_normal((n, ci))
    W = rng.standard_normal((5, ci, co))
    dP = rng.standard_normal((n, co))
    lhs = np.sum(nn.conv(H, W) * dP)
    assert np.isclose(lhs, np.sum(H * nn.conv_input_grad(dP, W)), rtol=1e-12)
    dW, db = nn.conv_weight_grad(H, dP, 5)
    assert np.isclose(lhs, np.sum(W * dW), rtol=1e-12)
    assert np.allclose(db, dP.sum(axis=0))


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    width, ci0, taps = 4, 8, 5
    P = nn.n_params(width, ci0, taps)
    params = rng.standard_normal(P) * 0.5
    Xs = [rng.standard_normal((n, nn.N_FEAT)) for n in (6, 9, 3)]
    labels = rng.standard_normal(3)
    loss, grad = nn.loss_and_grad(params, Xs, labels, bf16=False)
    h = 1e-6
    num = np.zeros(P)
    for i in range(P):
        e = np.zeros(P)
        e[i] = h
        lp, _ = nn.loss_and_grad(params + e, Xs, labels, bf16=False)
        lm, _ = nn.loss_and_grad(params - e, Xs, labels, bf16=False)
        num[i] = (lp - lm) / (2 * h)
    assert np.allclose(grad, num, rtol=1e-5, atol=1e-7)
    # the loss is the MSE of the forward pass
    y = nn.forward(params, Xs, bf16=False)
    assert np.isclose(loss, np.mean((y - labels) ** 2), rtol=1e-12)


def test_head_closed_forms():
    rng = np.random.default_rng(4)
    p = nn.unpack(rng.standard_normal(nn.n_params()) * 0.1)
    X = rng.standard_normal((7, nn.N_FEAT))
    # conv outputs all clipped to zero: z = 0, y = wb . relu(ba) + bb
    for l in range(1, 5):
        p[f"b{l}"] = np.full(nn.WIDTH, -1e3)
    y = nn.forward(nn.pack(p), [X], bf16=False)[0]
    assert np.isclose(y, p["wb"] @ np.maximum(p["ba"], 0) + p["bb"][0], rtol=1e-12)
    # zero conv weights, positive biases: H_l = b_l at every position, z = b4
    for l in range(1, 5):
        p[f"W{l}"] = np.zeros_like(p[f"W{l}"])
        p[f"b{l}"] = rng.uniform(0.1, 1.0, nn.WIDTH)
    y = nn.forward(nn.pack(p), [X], bf16=False)[0]
    want = p["wb"] @ np.maximum(p["Wa"] @ p["b4"] + p["ba"], 0) + p["bb"][0]
    assert np.isclose(y, want, rtol=1e-12)


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-2, 1e-8
    p1, m, v = nn.adam(p0, np.zeros(50), np.zeros(50), g, 1, lr, eps=eps)
    # bias correction makes the first step lr * g / (|g| + eps)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)
    # a constant gradient keeps that step size
    p2, _, _ = nn.adam(p1, m, v, g, 2, lr, eps=eps)
    assert np.allclose(p2, p1 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)


def test_features_of_a_hand_example():
    xy = np.array([[1, 1], [4, 5], [7, 9], [1, 6]])  # depot, customers 1..3
    d = np.array([[0, 5, 10, 5], [5, 0, 5, 3], [10, 5, 0, 7], [5, 3, 7, 0]])
    demand = np.array([[2, 4, 6, 8], [5, 5, 5, 5], [0, 10, 0, 10]], dtype=np.int16)
    mu, sd = nn.demand_stats(demand)
    assert np.allclose(mu, [5, 5, 5]) and np.allclose(sd, [np.sqrt(5), 0, 5])
    X = nn.features([2, 1, 3], d, mu, sd, Q=10, L=10.0, xy=xy)
    want = np.array([
        # dx   dy   mean  std            prev  next  depot  1
        [0.6, 0.8, 0.5, 0.0,            1.0,  0.5,  1.0,  1],
        [0.3, 0.4, 0.5, np.sqrt(5) / 10, 0.5, 0.3,  0.5,  1],
        [0.0, 0.5, 0.5, 0.5,            0.3,  0.5,  0.5,  1],
    ])
    assert np.allclose(X, want, atol=1e-15)
    # no coordinates (distance-matrix instance): the coordinate features are zero
    assert np.allclose(nn.features([2, 1, 3], d, mu, sd, 10, 10.0)[:, :2], 0)


def test_bf16_forward_stays_near_float64():
    rng = np.random.default_rng(6)
    params = rng.standard_normal(nn.n_params()) * 0.05
    Xs = [rng.uniform(0, 1, (40, nn.N_FEAT)) for _ in range(2)]
    y64 = nn.forward(params, Xs, bf16=False)
    y16 = nn.forward(params, Xs, bf16=True)
    assert np.all(np.abs(y16 - y64) <= 0.05 * (np.abs(y64) + 0.1))
