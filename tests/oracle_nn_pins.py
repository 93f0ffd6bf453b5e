"""Pins of the float64 surrogate reference (oracle/nn.py) against things other than itself:
numpy's correlation for the conv orientation and padding, adjoint identities for the two
backward convolutions, central finite differences for the whole float64 gradient, torch's
automatic differentiation (through torch's own conv1d) for the gradient with the bfloat16
rounding points, closed forms for the pooling/MLP head and for Adam's first steps, bit-level
float32 rounding for bfloat16, and a hand-computed feature table. CPU only.

Every pin takes the module under test, so that the same pins run against the reference and
against copies of it with planted mistakes."""
import numpy as np


def pin_bf16_round(m):
    rng = np.random.default_rng(0)
    x32 = (rng.standard_normal(20000) * np.exp(rng.uniform(-10, 10, 20000))).astype(np.float32)
    bits = x32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32).view(np.float32)
    assert np.array_equal(m.bf16_round(x32.astype(np.float64)), rounded.astype(np.float64))
    # ties go to the even significand
    assert m.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert m.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert m.bf16_round(-(1.0 + 3 * 2.0 ** -8)) == -(1.0 + 2.0 ** -6)


def pin_conv_is_numpy_correlate(m):
    rng = np.random.default_rng(1)
    for n in (1, 2, 5, 13):
        x = rng.standard_normal(n)
        w = rng.standard_normal(5)
        got = m.conv(x[:, None], w[:, None, None])[:, 0]
        # full correlation at lags -2 .. n-3 (numpy's "same" when n >= 5)
        want = np.correlate(x, w, mode="full")[2:2 + n]
        assert np.allclose(got, want, atol=1e-12, rtol=0)
        if n >= 5:
            assert np.allclose(got, np.correlate(x, w, mode="same"), atol=1e-12, rtol=0)


def pin_backward_convs_are_adjoints(m):
    rng = np.random.default_rng(2)
    n, ci, co = 11, 6, 7
    H = rng.standard_normal((n, ci))
    W = rng.standard_normal((5, ci, co))
    dP = rng.standard_normal((n, co))
    lhs = np.sum(m.conv(H, W) * dP)
    assert np.isclose(lhs, np.sum(H * m.conv_input_grad(dP, W)), rtol=1e-12)
    dW, db = m.conv_weight_grad(H, dP, 5)
    assert np.isclose(lhs, np.sum(W * dW), rtol=1e-12)
    assert np.allclose(db, dP.sum(axis=0))


def pin_gradient_central_differences(m):
    rng = np.random.default_rng(3)
    width, ci0, taps = 4, 8, 5
    P = m.n_params(width, ci0, taps)
    params = rng.standard_normal(P) * 0.5
    Xs = [rng.standard_normal((n, m.N_FEAT)) for n in (6, 9, 3)]
    labels = rng.standard_normal(3)
    loss, grad = m.loss_and_grad(params, Xs, labels, bf16=False)
    h = 1e-6
    num = np.zeros(P)
    for i in range(P):
        e = np.zeros(P)
        e[i] = h
        lp, _ = m.loss_and_grad(params + e, Xs, labels, bf16=False)
        lm, _ = m.loss_and_grad(params - e, Xs, labels, bf16=False)
        num[i] = (lp - lm) / (2 * h)
    assert np.allclose(grad, num, rtol=1e-5, atol=1e-7)
    # the loss is the MSE of the forward pass
    y = m.forward(params, Xs, bf16=False)
    assert np.isclose(loss, np.mean((y - labels) ** 2), rtol=1e-12)


def _bf16_torch(x):
    """bfloat16 rounding of float64 torch values through torch's own float32 -> bfloat16 cast.
    The float64 -> float32 step first rounds to 24 significant bits; it changes the final result
    only for a value whose bits 9 to 24 round to exactly one half of a bfloat16 unit, which the
    seeded inputs of the pin below never produce."""
    import torch
    return x.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _autograd_loss_and_grad(params, Xs, labels, width, ci0, taps):
    """The surrogate's loss and gradient by torch autograd through torch.nn.functional.conv1d,
    with the bfloat16 rounding points the model defines: inputs, conv weights and every H_l in
    the forward pass (straight through for the gradient), and every pre-activation gradient
    dP_l in the backward pass (a tensor hook)."""
    import torch
    import torch.nn.functional as F

    def rnd_st(x):  # rounded value, identity gradient
        return x + (_bf16_torch(x.detach()) - x.detach())

    flat = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    shapes = [("W1", (taps, ci0, width)), ("b1", (width,))]
    for l in (2, 3, 4):
        shapes += [(f"W{l}", (taps, width, width)), (f"b{l}", (width,))]
    shapes += [("Wa", (width, width)), ("ba", (width,)), ("wb", (width,)), ("bb", (1,))]
    p, off = {}, 0
    for name, shape in shapes:
        size = int(np.prod(shape))
        p[name] = flat[off:off + size].reshape(shape)
        off += size
    assert off == flat.numel()
    loss = torch.zeros((), dtype=torch.float64)
    T = len(Xs)
    for X, lab in zip(Xs, labels):
        n = X.shape[0]
        H = torch.zeros((n, ci0), dtype=torch.float64)
        H[:, :X.shape[1]] = torch.tensor(X)
        H = _bf16_torch(H)
        for l in range(1, 5):
            W = rnd_st(p[f"W{l}"])                         # [taps, CI, CO]
            Pre = F.conv1d(H.t()[None], W.permute(2, 1, 0), padding=(taps - 1) // 2)[0].t()
            Pre = Pre + p[f"b{l}"]
            Pre.register_hook(_bf16_torch)                 # dP_l rounded in the backward pass
            H = rnd_st(torch.relu(Pre))
        z = H.mean(dim=0)
        u = torch.relu(p["Wa"] @ z + p["ba"])
        y = p["wb"] @ u + p["bb"][0]
        loss = loss + (y - float(lab)) ** 2 / T
    loss.backward()
    return float(loss.detach()), flat.grad.numpy()


def pin_bf16_gradient_autograd(m):
    rng = np.random.default_rng(7)
    for width, ci0, taps, scale in ((8, 8, 5, 0.4), (16, 8, 3, 0.3)):
        P = m.n_params(width, ci0, taps)
        params = rng.standard_normal(P) * scale
        Xs = [rng.uniform(-1, 1, (n, m.N_FEAT)) for n in (7, 12, 2)]
        labels = rng.standard_normal(3)
        loss, grad = m.loss_and_grad(params, Xs, labels, bf16=True)
        loss_t, grad_t = _autograd_loss_and_grad(params, Xs, labels, width, ci0, taps)
        assert np.isclose(loss, loss_t, rtol=1e-10, atol=1e-12)
        assert np.allclose(grad, grad_t, rtol=1e-9, atol=1e-11 * np.abs(grad_t).max())
        # the forward pass agrees with the autograd graph's as well
        y = m.forward(params, Xs, bf16=True)
        assert np.isclose(np.mean((y - labels) ** 2), loss_t, rtol=1e-10, atol=1e-12)


def pin_head_closed_forms(m):
    rng = np.random.default_rng(4)
    p = m.unpack(rng.standard_normal(m.n_params()) * 0.1)
    X = rng.standard_normal((7, m.N_FEAT))
    # conv outputs all clipped to zero: z = 0, y = wb . relu(ba) + bb
    for l in range(1, 5):
        p[f"b{l}"] = np.full(m.WIDTH, -1e3)
    y = m.forward(m.pack(p), [X], bf16=False)[0]
    assert np.isclose(y, p["wb"] @ np.maximum(p["ba"], 0) + p["bb"][0], rtol=1e-12)
    # zero conv weights, positive biases: H_l = b_l at every position, z = b4
    for l in range(1, 5):
        p[f"W{l}"] = np.zeros_like(p[f"W{l}"])
        p[f"b{l}"] = rng.uniform(0.1, 1.0, m.WIDTH)
    y = m.forward(m.pack(p), [X], bf16=False)[0]
    want = p["wb"] @ np.maximum(p["Wa"] @ p["b4"] + p["ba"], 0) + p["bb"][0]
    assert np.isclose(y, want, rtol=1e-12)


def pin_adam_first_steps(m):
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-2, 1e-8
    p1, mm, v = m.adam(p0, np.zeros(50), np.zeros(50), g, 1, lr, eps=eps)
    # bias correction makes the first step lr * g / (|g| + eps)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)
    # a constant gradient keeps that step size
    p2, _, _ = m.adam(p1, mm, v, g, 2, lr, eps=eps)
    assert np.allclose(p2, p1 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)


def pin_features_hand_example(m):
    xy = np.array([[1, 1], [4, 5], [7, 9], [1, 6]])  # depot, customers 1..3
    d = np.array([[0, 5, 10, 5], [5, 0, 5, 3], [10, 5, 0, 7], [5, 3, 7, 0]])
    demand = np.array([[2, 4, 6, 8], [5, 5, 5, 5], [0, 10, 0, 10]], dtype=np.int16)
    mu, sd = m.demand_stats(demand)
    assert np.allclose(mu, [5, 5, 5]) and np.allclose(sd, [np.sqrt(5), 0, 5])
    X = m.features([2, 1, 3], d, mu, sd, Q=10, L=10.0, xy=xy)
    want = np.array([
        # dx   dy   mean  std            prev  next  depot  1
        [0.6, 0.8, 0.5, 0.0,            1.0,  0.5,  1.0,  1],
        [0.3, 0.4, 0.5, np.sqrt(5) / 10, 0.5, 0.3,  0.5,  1],
        [0.0, 0.5, 0.5, 0.5,            0.3,  0.5,  0.5,  1],
    ])
    assert np.allclose(X, want, atol=1e-15)
    # no coordinates (distance-matrix instance): the coordinate features are zero
    assert np.allclose(m.features([2, 1, 3], d, mu, sd, 10, 10.0)[:, :2], 0)


def pin_bf16_forward_near_float64(m):
    rng = np.random.default_rng(6)
    params = rng.standard_normal(m.n_params()) * 0.05
    Xs = [rng.uniform(0, 1, (40, m.N_FEAT)) for _ in range(2)]
    y64 = m.forward(params, Xs, bf16=False)
    y16 = m.forward(params, Xs, bf16=True)
    assert np.all(np.abs(y16 - y64) <= 0.05 * (np.abs(y64) + 0.1))


ALL_NN_PINS = [pin_bf16_round, pin_conv_is_numpy_correlate, pin_backward_convs_are_adjoints,
               pin_gradient_central_differences, pin_bf16_gradient_autograd,
               pin_head_closed_forms, pin_adam_first_steps, pin_features_hand_example,
               pin_bf16_forward_near_float64]
