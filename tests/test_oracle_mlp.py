"""Pins of the run-time-model oracle: gradients against central finite
differences, a closed-form case, and Adam's first step."""
import numpy as np

from oracle import mlp_ref
from paper_1710_01839_amd import inputs


def _data(R=40, F=14, seed=0):
    g = np.random.default_rng(seed)
    X = g.uniform(-1, 1, size=(R, F))
    t = g.normal(size=R)
    return X, t


def _params(F=14, H=16, seed=1):
    g = np.random.default_rng(seed)
    return {"W1": g.normal(0, 0.5, (H, F)), "b1": g.normal(0, 0.1, H),
            "W2": g.normal(0, 0.3, (H, H)), "b2": g.normal(0, 0.1, H),
            "W3": g.normal(0, 0.3, (1, H)), "b3": g.normal(0, 0.1, 1)}


def test_gradients_match_finite_differences():
    X, t = _data()
    P = _params()
    loss, g = mlp_ref.loss_and_grads(P, X, t)
    flat = mlp_ref.flatten(P)
    gflat = mlp_ref.flatten(g)
    rng = np.random.default_rng(2)
    h = 1e-6
    for idx in rng.choice(flat.size, size=60, replace=False):
        e = np.zeros_like(flat)
        e[idx] = h
        lp, _ = mlp_ref.loss_and_grads(mlp_ref.unflatten(flat + e, 14, 16), X, t)
        lm, _ = mlp_ref.loss_and_grads(mlp_ref.unflatten(flat - e, 14, 16), X, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[idx]) <= 1e-6 * max(1.0, abs(fd)), idx


def test_linear_case_closed_form():
    """With positive pre-activations the network is linear; the gradient of b3
    is 2 mean(y - t) and a zero residual gives zero gradients."""
    F, H = 3, 4
    P = {"W1": np.eye(H, F), "b1": np.full(H, 5.0), "W2": np.eye(H), "b2": np.ones(H),
         "W3": np.ones((1, H)), "b3": np.zeros(1)}
    X = np.array([[0.1, 0.2, 0.3], [0.0, -0.1, 0.2]])
    y, _ = mlp_ref.forward(P, X)
    assert np.allclose(y, [X[0].sum() + 4 * 6.0, X[1].sum() + 4 * 6.0])
    loss, g = mlp_ref.loss_and_grads(P, X, y)
    assert loss == 0.0 and all(np.all(v == 0) for v in g.values())
    loss, g = mlp_ref.loss_and_grads(P, X, y - 1.0)
    assert np.isclose(g["b3"][0], 2.0)


def test_adam_first_step_is_signed_lr():
    """Adam's first update is -lr * g / (|g| + eps') elementwise (bias
    corrections cancel)."""
    X, t = _data(seed=3)
    P = _params(seed=4)
    _, g = mlp_ref.loss_and_grads(P, X, t)
    P1, losses = mlp_ref.adam_train(P, X, t, 1, lr=1e-2)
    for k in mlp_ref.ORDER:
        step = P1[k] - P[k]
        assert np.allclose(step, -1e-2 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-9, atol=1e-15)


def test_training_reduces_loss_and_init_shapes():
    P = {k: v.astype(np.float64) for k, v in inputs.mlp_init(14, 64).items()}
    assert P["W1"].shape == (64, 14) and P["W3"].shape == (1, 64)
    X, t = _data(R=200, seed=5)
    t = X[:, 0] * 2 - X[:, 1] + 0.5
    _, losses = mlp_ref.adam_train(P, X, t, 200, lr=3e-3)
    assert losses[-1] < 0.1 * losses[0]
