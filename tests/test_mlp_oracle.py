"""The surrogate-network oracle against its pins, and broken copies against them (CPU)."""
import importlib.util
import os

import pytest

import oracle.mlp as MLP
from tests.mlp_pins import PINS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin(MLP)


# Plausible mistakes; each must fail at least one pin.
MUTANTS = {
    "gelu_d_uses_gelu": ("dZ2 = np.outer(dy_sum, r(w3)) * gelu_d(a[\"Z2\"])",
                         "dZ2 = np.outer(dy_sum, r(w3)) * gelu(a[\"Z2\"])"),
    "dropped_b2": ("Z2 = r(H1) @ r(W2).T + b2", "Z2 = r(H1) @ r(W2).T"),
    "transposed_W2_backward": ("dZ1 = (r(dZ2) @ r(W2)) * gelu_d(a[\"Z1\"])",
                               "dZ1 = (r(dZ2) @ r(W2).T) * gelu_d(a[\"Z1\"])"),
    "no_bias_correction": ("mh = m / (1.0 - b1 ** t)", "mh = m"),
    "gelu_tanh_form": ("return 0.5 * x * (1.0 + erf(x * _SQRT1_2))",
                       "return 0.5 * x * (1.0 + np.tanh(0.7978845608 * (x + 0.044715 * x ** 3)))"),
    "loss_not_mean": ("G = pack(dW1, db1, dW2, db2, dw3, db3) / B", "G = pack(dW1, db1, dW2, db2, dw3, db3)"),
    "features_no_norm": ("C = V * ph / np.where(nrm > 0, nrm, 1.0)", "C = V * ph"),
    "features_conj_phase": ("ph = np.exp(-1j * np.angle(V[:, :1]))", "ph = np.exp(1j * np.angle(V[:, :1]))"),
    "targets_no_log": ("t[fin] = np.log1p(nll[fin] - lo)", "t[fin] = nll[fin] - lo"),
    "topk_ties_reversed": ("order = np.lexsort((np.arange(keys.shape[0]), keys))",
                           "order = np.lexsort((-np.arange(keys.shape[0]), keys))"),
    "round_result_not_operand": ("Z1 = r(X) @ r(W1).T + b1", "Z1 = r(X @ W1.T) + b1"),
    "f16_truncates": ("return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float16)",
                      "return np.trunc(np.asarray(x, dtype=np.float64) * 1024) / 1024 + 0 * np.asarray(x).astype(np.float16)"),
}


def _mutant(name):
    src = open(os.path.join(ROOT, "oracle", "mlp.py")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    spec = importlib.util.spec_from_loader(f"mlp_mutant_{name}", loader=None)
    mod = importlib.util.module_from_spec(spec)
    exec(compile(src.replace(old, new), f"<mutant {name}>", "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    M = _mutant(name)
    caught = []
    for pin in PINS:
        try:
            pin(M)
        except Exception:
            caught.append(pin.__name__)
    assert caught, f"mutant {name} passes every pin"
