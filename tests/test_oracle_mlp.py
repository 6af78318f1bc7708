"""Pins for the FP64 reference of the order-selection network and its
training data (CPU only), and planted mistakes they must catch.

Pins: central finite differences of the loss (a textbook check of any
backward pass); the closed form of the output-bias gradient; the affine
network the model reduces to when every ReLU is active; and, for the
training data, the exact zero error of order 10 against itself, the decay
of the truncation error with the order, and the closed-form features of a
point charge at the cell centre.
"""
import importlib.util
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from oracle import mlp  # noqa: E402


def pin_finite_differences(m):
    rng = np.random.default_rng(5)
    theta = m.init_params(3) + 0.05 * rng.standard_normal(m.NPARAM)
    X = rng.standard_normal((23, m.NIN))
    T = rng.standard_normal((23, m.NOUT))
    g = m.grad(theta, X, T)
    idx = rng.choice(m.NPARAM, 120, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(m.NPARAM)
        e[i] = h
        fd = (m.loss(theta + e, X, T) - m.loss(theta - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, g[i])


def pin_output_bias_closed_form(m):
    """d/db3_k mean((Y - T)^2) = 2 sum_b (Y_bk - T_bk) / (9 B)."""
    rng = np.random.default_rng(6)
    theta = m.init_params(4)
    X = rng.standard_normal((17, m.NIN))
    T = rng.standard_normal((17, m.NOUT))
    Y, _ = m.forward(theta, X)
    g = m.grad(theta, X, T)
    want = 2.0 * (Y - T).sum(axis=0) / (9 * 17)
    assert np.allclose(g[-m.NOUT:], want, rtol=1e-12, atol=1e-15)


def pin_affine_when_relus_active(m):
    """Large positive hidden biases keep every ReLU active: the network is
    then the affine map y = W3 (W2 (W1 x + b1) + b2) + b3."""
    rng = np.random.default_rng(7)
    W1 = 0.01 * rng.standard_normal((m.NH, m.NIN)); b1 = np.full(m.NH, 50.0)
    W2 = 0.01 * rng.standard_normal((m.NH, m.NH)); b2 = np.full(m.NH, 50.0)
    W3 = 0.1 * rng.standard_normal((m.NOUT, m.NH)); b3 = rng.standard_normal(m.NOUT)
    theta = np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])
    X = rng.standard_normal((9, m.NIN))
    Y, (_, Z1, _, Z2, _) = m.forward(theta, X)
    assert np.all(Z1 > 0) and np.all(Z2 > 0)
    want = np.array([W3 @ (W2 @ (W1 @ x + b1) + b2) + b3 for x in X])
    assert np.allclose(Y, want, rtol=1e-12, atol=1e-12)


def _cluster_multipole(seed, n=30):
    rng = np.random.default_rng(seed)
    src = rng.uniform(-0.5, 0.5, (n, 3))
    q = rng.uniform(0.5, 1.5, n)
    return oracle.p2m(10, np.zeros(3), src, q)


def pin_labels(m):
    M = _cluster_multipole(8)
    for v in ((2, 0, 0), (2, 2, 1), (3, -3, 3)):
        y = m.truncation_labels(M, v)
        assert y.shape == (9,) and y[-1] == -15.0, y
        # the truncation error falls with the order (well-separated pair)
        assert all(b < a for a, b in zip(y[:-2], y[1:-1])), (v, y)
    # a farther target converges faster at every order below 10
    yn, yf = m.truncation_labels(M, (2, 0, 0)), m.truncation_labels(M, (3, 3, 3))
    assert np.all(yf[:-1] < yn[:-1])


def pin_features_point_charge(m):
    """A charge q at the cell centre: only the rank-0 component is non-zero."""
    M = oracle.p2m(10, np.zeros(3), np.zeros((1, 3)), np.array([2.5]))
    x = m.features(M, (2, 1, 0))
    assert abs(x[0] - np.sqrt(5.0) / (np.sqrt(3.0) / 2.0)) < 1e-15
    assert x[1] == 0.0 and np.all(x[2:] < -250.0)


PINS = [pin_finite_differences, pin_output_bias_closed_form, pin_affine_when_relus_active, pin_labels,
        pin_features_point_charge]


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin(mlp)


MUTANTS = [
    ("relu_mask_dropped", "dZ2 = (dY @ W3) * (Z2 > 0.0)", "dZ2 = (dY @ W3)"),
    ("loss_factor_two", "dY = 2.0 * (Y - T) / Y.size", "dY = (Y - T) / Y.size"),
    ("wrong_layer_input", "gW2 = dZ2.T @ H1", "gW2 = dZ2.T @ Z1"),
    ("bias_sum_axis", "gb1 = dZ1.sum(axis=0)", "gb1 = dZ1.mean(axis=0)"),
    ("label_reference_order", "ref = fields[10]", "ref = fields[9]"),
    ("feature_radius", "x[0] = np.sqrt(float(np.dot(v, v))) / (np.sqrt(3.0) / 2.0)",
     "x[0] = np.sqrt(float(np.dot(v, v)))"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, old, new):
    src = open(os.path.join(ROOT, "oracle", "mlp.py")).read()
    assert old in src
    path = tmp_path / f"mlp_{name}.py"
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"mlp_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    failed = []
    for pin in PINS:
        try:
            pin(mod)
        except AssertionError:
            failed.append(pin.__name__)
    assert failed, f"no pin rejects mutant {name}"
