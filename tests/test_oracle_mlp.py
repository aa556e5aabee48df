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


def test_adam_later_steps_closed_form():
    """Adam (Kingma and Ba, Alg. 1; beta1 = 0.9, beta2 = 0.999) on the gradient sequence
    g, 0, 0: after the first step the bias-corrected moments are geometric averages in
    closed form, m_hat_t = b1^(t-1) (1 - b1) / (1 - b1^t) g and
    v_hat_t = b2^(t-1) (1 - b2) / (1 - b2^t) g^2, so step t moves the weight by
    lr m_hat_t / (sqrt(v_hat_t) + eps).  With g = 1 the step factors are
    0.9/1.9 / sqrt(0.999/1.999) at t = 2 and 0.81/2.71 / sqrt(0.998001/2.997001) at t = 3
    (the two betas in swapped roles would give 0.7261 and 0.7779)."""
    lr, eps = 1e-2, 1e-8
    g = np.array([1.0, -4.0])
    w = np.array([0.3, 0.7])
    m = np.zeros(2); v = np.zeros(2)
    w1, m, v = mlp.adam(w, g, m, v, 1, lr)
    w2, m, v = mlp.adam(w1, np.zeros(2), m, v, 2, lr)
    w3, m, v = mlp.adam(w2, np.zeros(2), m, v, 3, lr)
    f2 = (0.9 / 1.9) / (np.sqrt(0.999 / 1.999) + eps)
    f3 = (0.81 / 2.71) / (np.sqrt(0.998001 / 2.997001) + eps)
    np.testing.assert_allclose(w1 - w, -lr * np.sign(g), rtol=1e-7)
    np.testing.assert_allclose(w2 - w1, -lr * np.sign(g) * np.array([f2, (0.9 / 1.9) / (np.sqrt(0.999 / 1.999) + eps / 4)]), rtol=1e-9)
    np.testing.assert_allclose(w3 - w2, -lr * np.sign(g) * np.array([f3, (0.81 / 2.71) / (np.sqrt(0.998001 / 2.997001) + eps / 4)]), rtol=1e-9)
    assert abs(f2 - 0.6700) < 1e-3 and abs(f3 - 0.5180) < 1e-3


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
