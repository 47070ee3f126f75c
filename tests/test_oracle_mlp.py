"""Pins of the cost-model MLP oracle: central finite differences for every
gradient, closed-form special cases, and properties of Adam that follow from
its definition (Kingma and Ba 2015) rather than from retyping it."""
import numpy as np
import pytest

from oracle import mlp


@pytest.fixture(scope="module")
def setup():
    g = np.random.default_rng(99)
    p = mlp.init_params(g)
    p["b1"] = g.standard_normal(mlp.N_HID) * 0.1
    p["b2"] = g.standard_normal(mlp.N_OUT) * 0.1
    X = g.standard_normal((7, mlp.N_IN))
    T = g.standard_normal((7, mlp.N_OUT))
    Mk = (g.random((7, mlp.N_OUT)) < 0.8).astype(np.float64)
    return p, X, T, Mk


def test_gradients_match_central_differences(setup):
    p, X, T, Mk = setup
    Y, cache = mlp.forward(p, X)
    g = mlp.backward(p, cache, Y, T, Mk)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2"):
        fd = np.zeros_like(p[name])
        it = np.nditer(p[name], flags=["multi_index"])
        for _ in it:
            ix = it.multi_index
            old = p[name][ix]
            p[name][ix] = old + h
            lp = mlp.loss(mlp.forward(p, X)[0], T, Mk)
            p[name][ix] = old - h
            lm = mlp.loss(mlp.forward(p, X)[0], T, Mk)
            p[name][ix] = old
            fd[ix] = (lp - lm) / (2 * h)
        err = np.linalg.norm(fd - g[name]) / max(np.linalg.norm(g[name]), 1e-30)
        assert err < 1e-6, (name, err)


def test_zero_weights_give_bias_output_and_zero_first_layer_gradient():
    g = np.random.default_rng(3)
    p = {"W1": np.zeros((32, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": g.standard_normal(64)}
    X = g.standard_normal((5, 32))
    Y, cache = mlp.forward(p, X)
    assert np.array_equal(Y, np.broadcast_to(p["b2"], (5, 64)))
    gr = mlp.backward(p, cache, Y, np.zeros((5, 64)), np.ones((5, 64)))
    assert np.all(gr["W1"] == 0) and np.all(gr["W2"] == 0) and np.all(gr["b1"] == 0)
    # d/db2 of mean squared error with target 0 is 2*b2/64 per output (mean over 5*64 entries, 5 rows)
    assert np.allclose(gr["b2"], 2.0 * p["b2"] * 5 / (5 * 64))


def test_single_hidden_unit_hand_gradient():
    # one active hidden unit, one input, one output weight: L = (w2*(w1*x) - t)^2 over one entry
    p = {"W1": np.zeros((32, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64)}
    p["W1"][0, 0] = 0.5
    p["W2"][0, 0] = 3.0
    X = np.zeros((1, 32))
    X[0, 0] = 2.0
    T = np.zeros((1, 64))
    T[0, 0] = 1.0
    Mk = np.zeros((1, 64))
    Mk[0, 0] = 1.0
    Y, cache = mlp.forward(p, X)
    assert Y[0, 0] == 3.0  # 3 * relu(0.5*2)
    gr = mlp.backward(p, cache, Y, T, Mk)
    r = 3.0 - 1.0
    assert gr["W2"][0, 0] == 2 * r * 1.0       # dL/dw2 = 2 r h, h = 1
    assert gr["W1"][0, 0] == 2 * r * 3.0 * 2.0  # dL/dw1 = 2 r w2 x
    assert gr["b2"][0] == 2 * r


def test_adam_first_step_is_lr_times_sign():
    g = np.random.default_rng(5)
    w = g.standard_normal(100)
    grad = g.standard_normal(100)
    m, v = np.zeros(100), np.zeros(100)
    w0 = w.copy()
    mlp.adam_step(w, grad, m, v, 1, lr=1e-2)
    assert np.allclose(w0 - w, 1e-2 * np.sign(grad), rtol=1e-6)


def test_adam_constant_gradient_keeps_step():
    w = np.array([1.0, -2.0])
    grad = np.array([0.3, -4.0])
    m, v = np.zeros(2), np.zeros(2)
    for t in range(1, 50):
        prev = w.copy()
        mlp.adam_step(w, grad, m, v, t, lr=1e-3)
        # bias correction makes mhat = g and vhat = g^2 for a constant gradient
        assert np.allclose(prev - w, 1e-3 * grad / (np.abs(grad) + 1e-8), rtol=1e-9)


def test_training_reduces_loss():
    g = np.random.default_rng(11)
    p = mlp.init_params(g)
    X = g.standard_normal((256, 32))
    Wt = g.standard_normal((32, 64)) * 0.3
    T = X @ Wt
    Mk = np.ones_like(T)
    st = {k: (np.zeros_like(v), np.zeros_like(v)) for k, v in p.items()}
    l0 = mlp.loss(mlp.forward(p, X)[0], T, Mk)
    for t in range(1, 301):
        Y, cache = mlp.forward(p, X)
        gr = mlp.backward(p, cache, Y, T, Mk)
        for k in p:
            mlp.adam_step(p[k], gr[k], st[k][0], st[k][1], t, lr=3e-3)
    l1 = mlp.loss(mlp.forward(p, X)[0], T, Mk)
    assert l1 < 0.2 * l0
