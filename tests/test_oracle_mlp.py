"""Pins of the fp64 CDF-model oracle: finite differences for the gradient,
closed forms for forward and for the first Adam step."""
import numpy as np

from oracle import mlp


def _params(seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.5, mlp.N_PARAMS)


def test_param_count():
    assert mlp.N_PARAMS == 1153


def test_forward_closed_form():
    # W1 = 1, b1 = 0 -> h1 = relu(x) in every unit; W2 = I / 32, b2 = 0 ->
    # h2 = relu(x) / 32; W3 = 1, b3 = 0.25 -> y = relu(x) + 0.25
    p = np.zeros(mlp.N_PARAMS)
    o = 0
    p[o:o + 32] = 1.0
    o += 64
    p[o:o + 1024] = (np.eye(32) / 32.0).reshape(-1)
    o += 1024 + 32
    p[o:o + 32] = 1.0
    p[o + 32] = 0.25
    x = np.array([-1.0, 0.0, 0.5, 2.0])
    y, _ = mlp.forward(p, x)
    assert np.allclose(y, np.maximum(x, 0) + 0.25, rtol=0, atol=1e-15)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    p = _params(1)
    x = rng.uniform(0, 1, 64)
    t = np.sort(rng.uniform(0, 1, 64))
    L, g = mlp.backward(p, x, t)
    assert abs(L - mlp.loss(p, x, t)) < 1e-15
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False).tolist() + [0, 32, 64, 1088, 1120, 1152]
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, x, t) - mlp.loss(p - e, x, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g).max()), i


def test_first_adam_step_moves_each_parameter_by_lr():
    # after one step m_hat = g and v_hat = g^2, so each parameter moves by
    # lr * g / (|g| + eps): almost exactly lr against the sign of g
    rng = np.random.default_rng(4)
    p = _params(2)
    g = rng.normal(0, 1, mlp.N_PARAMS)
    p1, m, v = mlp.adam_step(p, np.zeros_like(p), np.zeros_like(p), g, step=1, lr=1e-3)
    # |lr * g / (|g| + eps) - lr * sign(g)| = lr * eps / (|g| + eps)
    err = np.abs((p - p1) - 1e-3 * np.sign(g))
    assert np.all(err <= 1e-3 * 1e-8 / np.abs(g) + 1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_keeps_step_size():
    # with a constant gradient the bias-corrected ratio stays 1: every step moves lr
    p = np.zeros(mlp.N_PARAMS)
    g = np.full(mlp.N_PARAMS, 0.3)
    m = v = np.zeros_like(p)
    for step in range(1, 6):
        p, m, v = mlp.adam_step(p, m, v, g, step=step, lr=0.01)
    assert np.allclose(p, -0.05, rtol=1e-6)


def test_training_fits_uniform_cdf():
    # the CDF of uniform keys on [0, 1] is the identity; a few hundred Adam
    # steps on a sorted sample must bring the loss well below its start
    rng = np.random.default_rng(5)
    x = np.sort(rng.uniform(0, 1, 512))
    t = np.arange(512) / 512.0
    p = _params(7) * 0.3
    m = v = np.zeros_like(p)
    L0 = mlp.loss(p, x, t)
    for step in range(1, 301):
        _, g = mlp.backward(p, x, t)
        p, m, v = mlp.adam_step(p, m, v, g, step=step, lr=3e-3)
    assert mlp.loss(p, x, t) < 0.05 * L0
