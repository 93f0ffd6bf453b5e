"""Plant plausible mistakes in copies of the float64 surrogate reference (oracle/nn.py) and
check that its pins catch every one: a transposed or mirrored tap, a padding row off by one, a
bfloat16 rounding dropped or moved, a wrong mask, a dropped bias correction. CPU only."""
import importlib.util
import os

import pytest

from oracle import nn
from oracle_nn_pins import ALL_NN_PINS

SRC = nn.__file__

# (name, exact text in oracle/nn.py, replacement)
MUTANTS = [
    ("conv_mirrored_taps", "        out += Hp[k:k + n] @ W[k]\n",
     "        out += Hp[k:k + n] @ W[taps - 1 - k]\n"),
    ("conv_padding_row", "    Hp[pad:pad + n] = H\n    out = np.zeros((n, W.shape[2]))",
     "    Hp[pad + 1:pad + 1 + n] = H\n    out = np.zeros((n, W.shape[2]))"),
    ("input_grad_tap_direction", "dH += dPp[2 * pad - k:2 * pad - k + n] @ W[k].T",
     "dH += dPp[k:k + n] @ W[k].T"),
    ("input_grad_untransposed", "dH += dPp[2 * pad - k:2 * pad - k + n] @ W[k].T",
     "dH += dPp[2 * pad - k:2 * pad - k + n] @ W[k]"),
    ("weight_grad_mirrored_taps", "dW = np.stack([Hp[k:k + n].T @ dP for k in range(taps)])",
     "dW = np.stack([Hp[taps - 1 - k:taps - 1 - k + n].T @ dP for k in range(taps)])"),
    ("weight_grad_padding_row", "    Hp[pad:pad + n] = H\n    dW = np.stack(",
     "    Hp[pad - 1:pad - 1 + n] = H\n    dW = np.stack("),
    ("backward_rounding_dropped", "dP = rnd(dH * (H[l - 1] > 0))", "dP = dH * (H[l - 1] > 0)"),
    ("pool_gradient_rounded_early",
     "dP = rnd(np.broadcast_to(dz / n, H[4].shape) * (H[4] > 0))",
     "dP = np.broadcast_to(rnd(dz) / n, H[4].shape) * (H[4] > 0)"),
    ("weights_not_rounded", 'Ws = [rnd(p[f"W{l}"]) for l in range(1, 5)]',
     'Ws = [p[f"W{l}"] for l in range(1, 5)]'),
    ("mask_from_wrong_layer", "dP = rnd(dH * (H[l - 1] > 0))", "dP = rnd(dH * (H[l] > 0))"),
    ("sum_pool", "z = H[4].mean(axis=0)", "z = H[4].sum(axis=0)"),
    ("adam_no_bias_correction", "mhat = m / (1.0 - beta1 ** step)", "mhat = m"),
    ("feature_next_arc", "X[j, 5] = float(d[c][nxt]) / L", "X[j, 5] = float(d[prev][c]) / L"),
    ("bf16_truncates", "return np.ldexp(np.round(m * 256.0), e - 8)",
     "return np.ldexp(np.trunc(m * 256.0), e - 8)"),
    ("population_std_with_ddof", "sd = np.sqrt(np.maximum((q * q).mean(axis=1) - mu * mu, 0.0))",
     "sd = np.sqrt(np.maximum((q * q).sum(axis=1) / max(q.shape[1] - 1, 1) - mu * mu, 0.0))"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    path = tmp_path / f"nn_{name}.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"nn_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = []
    for pin in ALL_NN_PINS:
        try:
            pin(mod)
        except (AssertionError, ValueError):
            caught.append(pin.__name__)
    print(f"{name}: caught by {caught}")
    assert caught, f"no pin caught mutant {name}"
