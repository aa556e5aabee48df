"""Pins of the MLP oracle: back-propagation against finite differences of the loss
(rounding off), bfloat16 rounding against torch's bfloat16 cast, Adam against its
published update, and a training run that lowers the loss."""
import numpy as np
import pytest

from oracle import mlp


def test_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(scale=s, size=2000) for s in (1e-3, 1.0, 1e3)])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), want)


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(1)
    vec = mlp.init_params(3) + rng.normal(scale=0.05, size=mlp.N_PARAMS)
    X = rng.normal(size=(17, mlp.N_IN))
    Y = rng.normal(size=(17, mlp.N_OUT))
    g, _ = mlp.grad(vec, X, Y, rounding=False)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS); e[i] = h
        fd = (mlp.loss(vec + e, X, Y, False) - mlp.loss(vec - e, X, Y, False)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_rounding_changes_little():
    rng = np.random.default_rng(2)
    vec = mlp.init_params(4)
    X = rng.normal(size=(64, mlp.N_IN)); Y = rng.normal(size=(64, mlp.N_OUT))
    g0, _ = mlp.grad(vec, X, Y, rounding=False)
    g1, _ = mlp.grad(vec, X, Y, rounding=True)
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 3e-2


def test_adam_step():
    w = np.array([1.0, -2.0]); g = np.array([0.5, -0.25])
    w1, m, v = mlp.adam(w, g, np.zeros(2), np.zeros(2), 1, 1e-2)
    # first step moves each weight by lr against the gradient's sign
    np.testing.assert_allclose(w1, w - 1e-2 * np.sign(g), rtol=1e-6)


def test_training_lowers_loss():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(512, mlp.N_IN))
    A = rng.normal(size=(mlp.N_IN, mlp.N_OUT)) * 0.3
    Y = np.tanh(X @ A)
    vec = mlp.init_params(6)
    m = np.zeros_like(vec); v = np.zeros_like(vec)
    l0 = mlp.loss(vec, X, Y)
    for t in range(1, 201):
        b = rng.choice(512, 64, replace=False)
        g, _ = mlp.grad(vec, X[b], Y[b])
        vec, m, v = mlp.adam(vec, g, m, v, t, 3e-3)
    assert mlp.loss(vec, X, Y) < 0.3 * l0
