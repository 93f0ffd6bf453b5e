"""Float64 reference of the tour-encoder surrogate -- TEST INFRASTRUCTURE ONLY.

The surrogate predicts a giant tour's expected second-stage cost (the sample mean of f(n) over
the scenarios, Section 2's two-stage objective evaluated by Section 3's Split) from features
along the tour. It is not part of the paper; its definition here is the one the GPU library
implements, written plainly in numpy float64 with explicit loops over taps:

  features of position j (tour s_1..s_n, depot 0, length scale L, capacity Q):
    x(s_j) - x(0), y(s_j) - y(0)             (divided by L; 0 for distance-matrix instances)
    mean and population std of s_j's demand   (over the scenarios, divided by Q)
    c(s_{j-1}, s_j), c(s_j, s_{j+1}), c(0, s_j)  (divided by L; s_0 = s_{n+1} = depot)
    1
  H_0 = features, zero-padded to 32 channels and by 2 positions on each side
  H_l = relu(conv_l(H_{l-1}) + b_l), l = 1..4, width 128, 5 taps:
        conv(H)[j] = sum_k H_pad[j + k] @ W[k]      (cross-correlation, "same" length)
  z = mean_j H_4[j];  u = relu(Wa z + ba);  y = wb . u + bb
  prediction = y * scale + shift               (label normalization of the model)

With bf16=True the values the GPU stores in bfloat16 are rounded to bfloat16 (nearest, ties to
even) at the same points: the input features, the conv weights, every H_l, and in the backward
pass every pre-activation gradient dP_l. All arithmetic between those points is float64.
Loss: mean over the batch of (y - label_norm)^2. Adam: the textbook update with bias
correction. Only tests/, the smoke check and the benchmark's CPU-baseline leg may import this
module; it imports nothing from the GPU library.
"""
from __future__ import annotations

import numpy as np

TAPS = 5
PAD = 2
N_FEAT = 8
CI0 = 32
WIDTH = 128


def param_shapes(width: int = WIDTH, ci0: int = CI0, taps: int = TAPS):
    """(name, shape) of every parameter, in the order of the flat parameter vector."""
    return [("W1", (taps, ci0, width)), ("b1", (width,)),
            ("W2", (taps, width, width)), ("b2", (width,)),
            ("W3", (taps, width, width)), ("b3", (width,)),
            ("W4", (taps, width, width)), ("b4", (width,)),
            ("Wa", (width, width)), ("ba", (width,)),
            ("wb", (width,)), ("bb", (1,))]


def n_params(width: int = WIDTH, ci0: int = CI0, taps: int = TAPS) -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes(width, ci0, taps))


def unpack(flat, width: int = WIDTH, ci0: int = CI0, taps: int = TAPS) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for name, shape in param_shapes(width, ci0, taps):
        size = int(np.prod(shape))
        out[name] = flat[off:off + size].reshape(shape)
        off += size
    assert off == flat.size, "parameter vector has the wrong length"
    return out


def pack(p: dict) -> np.ndarray:
    names = [n for n, _ in param_shapes(p["Wa"].shape[0], p["W1"].shape[1], p["W1"].shape[0])]
    return np.concatenate([np.asarray(p[n], dtype=np.float64).ravel() for n in names])


def bf16_round(x):
    """Nearest bfloat16 value (8 significant bits, ties to even) of float64 values."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)  # x = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)


def demand_stats(demand, S: int | None = None):
    """Mean and population standard deviation of every customer's demand over S scenarios."""
    q = np.asarray(demand)[:, :S].astype(np.float64)
    mu = q.mean(axis=1)
    sd = np.sqrt(np.maximum((q * q).mean(axis=1) - mu * mu, 0.0))
    return mu, sd


def features(tour, d, mu, sd, Q: int, L: float, xy=None) -> np.ndarray:
    """[n, 8] features of one tour (float64, before any rounding)."""
    tour = [int(c) for c in tour]
    n = len(tour)
    X = np.zeros((n, N_FEAT))
    for j, c in enumerate(tour):
        prev = tour[j - 1] if j > 0 else 0
        nxt = tour[j + 1] if j + 1 < n else 0
        if xy is not None:
            X[j, 0] = (float(xy[c][0]) - float(xy[0][0])) / L
            X[j, 1] = (float(xy[c][1]) - float(xy[0][1])) / L
        X[j, 2] = mu[c - 1] / Q
        X[j, 3] = sd[c - 1] / Q
        X[j, 4] = float(d[prev][c]) / L
        X[j, 5] = float(d[c][nxt]) / L
        X[j, 6] = float(d[0][c]) / L
        X[j, 7] = 1.0
    return X


def conv(H, W, b=None):
    """Cross-correlation over positions with 'same' length: out[j] = sum_k H_pad[j + k] @ W[k]
    (+ b), H [n, CI], W [taps, CI, CO], H_pad = H with (taps - 1) / 2 zero rows on each side."""
    taps = W.shape[0]
    pad = (taps - 1) // 2
    n = H.shape[0]
    Hp = np.zeros((n + 2 * pad, H.shape[1]))
    Hp[pad:pad + n] = H
    out = np.zeros((n, W.shape[2]))
    for k in range(taps):
        out += Hp[k:k + n] @ W[k]
    if b is not None:
        out += b
    return out


def conv_input_grad(dP, W):
    """Gradient of conv's input: dH[i] = sum_k dP[i - k + pad] @ W[k]^T (dP zero outside)."""
    taps = W.shape[0]
    pad = (taps - 1) // 2
    n = dP.shape[0]
    dPp = np.zeros((n + 2 * pad, dP.shape[1]))
    dPp[pad:pad + n] = dP
    dH = np.zeros((n, W.shape[1]))
    for k in range(taps):
        # position i receives dP[i - k + pad], which sits at padded row i - k + 2 pad
        dH += dPp[2 * pad - k:2 * pad - k + n] @ W[k].T
    return dH


def conv_weight_grad(H, dP, taps: int):
    """dW[k] = sum_j H_pad[j + k]^T dP[j] (outer products), and db = sum_j dP[j]."""
    pad = (taps - 1) // 2
    n = H.shape[0]
    Hp = np.zeros((n + 2 * pad, H.shape[1]))
    Hp[pad:pad + n] = H
    dW = np.stack([Hp[k:k + n].T @ dP for k in range(taps)])
    return dW, dP.sum(axis=0)


def _prep_input(X, ci0: int, bf16: bool):
    X = np.asarray(X, dtype=np.float64)
    H0 = np.zeros((X.shape[0], ci0))
    H0[:, :X.shape[1]] = X
    return bf16_round(H0) if bf16 else H0


def forward_one(p: dict, X, bf16: bool = True):
    """Forward pass of one tour's features X [n, 8]: y and the cache for backward."""
    rnd = bf16_round if bf16 else (lambda a: a)
    Ws = [rnd(p[f"W{l}"]) for l in range(1, 5)]
    H = [_prep_input(X, p["W1"].shape[1], bf16)]
    for l in range(4):
        H.append(rnd(np.maximum(conv(H[-1], Ws[l], p[f"b{l + 1}"]), 0.0)))
    z = H[4].mean(axis=0)
    a = p["Wa"] @ z + p["ba"]
    u = np.maximum(a, 0.0)
    y = float(p["wb"] @ u + p["bb"][0])
    return y, {"H": H, "Ws": Ws, "z": z, "a": a, "u": u}


def forward(params, Xs, bf16: bool = True) -> np.ndarray:
    """Normalized predictions y of a batch (Xs: list or array of [n, 8] features)."""
    p = unpack(params, *_dims(params))
    return np.array([forward_one(p, X, bf16)[0] for X in Xs])


def _dims(params):
    """(width, ci0, taps) of a flat parameter vector of one of the supported shapes."""
    for width, ci0 in ((WIDTH, CI0), (4, 8), (8, 8), (16, 8)):
        for taps in (TAPS, 3):
            if n_params(width, ci0, taps) == np.asarray(params).size:
                return width, ci0, taps
    raise ValueError("unsupported parameter vector length")


def loss_and_grad(params, Xs, labels, bf16: bool = True):
    """MSE loss of a batch and its gradient with respect to the flat parameter vector."""
    dims = _dims(params)
    p = unpack(params, *dims)
    T = len(Xs)
    labels = np.asarray(labels, dtype=np.float64)
    rnd = bf16_round if bf16 else (lambda a: a)
    g = {k: np.zeros_like(v) for k, v in p.items()}
    loss = 0.0
    for t in range(T):
        y, c = forward_one(p, Xs[t], bf16)
        err = y - labels[t]
        loss += err * err / T
        dy = 2.0 * err / T
        g["wb"] += dy * c["u"]
        g["bb"] += dy
        da = dy * p["wb"] * (c["a"] > 0)
        g["Wa"] += np.outer(da, c["z"])
        g["ba"] += da
        dz = p["Wa"].T @ da
        H = c["H"]
        n = H[4].shape[0]
        dP = rnd(np.broadcast_to(dz / n, H[4].shape) * (H[4] > 0))
        for l in range(4, 0, -1):
            dW, db = conv_weight_grad(H[l - 1], dP, dims[2])
            g[f"W{l}"] += dW
            g[f"b{l}"] += db
            if l > 1:
                dH = conv_input_grad(dP, c["Ws"][l - 1])
                dP = rnd(dH * (H[l - 1] > 0))
    return loss, pack(g)


def adam(params, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (step counts from 1). Returns (params, m, v)."""
    m = beta1 * np.asarray(m) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v) + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return np.asarray(params) - lr * mhat / (np.sqrt(vhat) + eps), m, v
