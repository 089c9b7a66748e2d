"""Pins of the FP64 MLP oracle: finite differences, closed forms, Adam."""
import numpy as np
import pytest

from oracle import mlp


def _setup(seed=0, B=7):
    params = mlp.init_params([8, 16, 16, 16, 2], seed)
    rng = np.random.default_rng(seed + 1)
    X = rng.standard_normal((B, 8))
    T = rng.standard_normal((B, 2))
    M = (rng.random((B, 2)) > 0.2).astype(float)
    return params, X, T, M


def test_gradients_match_finite_differences():
    params, X, T, M = _setup()
    g = mlp.gradients(params, X, T, M)
    h = 1e-6
    rng = np.random.default_rng(5)
    for li in range(len(params)):
        for which in (0, 1):
            P = params[li][which]
            for _ in range(6):
                idx = tuple(rng.integers(0, s) for s in P.shape)
                orig = P[idx]
                P[idx] = orig + h
                lp = mlp.loss(params, X, T, M)
                P[idx] = orig - h
                lm = mlp.loss(params, X, T, M)
                P[idx] = orig
                fd = (lp - lm) / (2 * h)
                assert g[li][which][idx] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_linear_layer_closed_form():
    """With one layer the model is affine: gradient = 2 (XW^T + b - T)^T X / count."""
    rng = np.random.default_rng(3)
    W, b = rng.standard_normal((2, 8)), rng.standard_normal(2)
    X, T = rng.standard_normal((5, 8)), rng.standard_normal((5, 2))
    M = np.ones((5, 2))
    gW, gb = mlp.gradients([(W, b)], X, T, M)[0]
    R = X @ W.T + b - T
    assert np.allclose(gW, 2 * R.T @ X / 10)
    assert np.allclose(gb, 2 * R.sum(axis=0) / 10)


def test_masked_outputs_get_no_gradient():
    params, X, T, M = _setup()
    M[:, 1] = 0.0
    g = mlp.gradients(params, X, T, M)
    assert np.all(g[-1][0][1] == 0) and g[-1][1][1] == 0


def test_adam_first_step_is_signed_lr():
    """After one step with zero state, Adam moves every parameter by lr*sign(g) (|g| >> eps)."""
    params, X, T, M = _setup()
    g = mlp.gradients(params, X, T, M)
    st = {}
    new = mlp.adam_step(params, g, st, lr=1e-3)
    for (W, b), (W2, b2), (gW, gb) in zip(params, new, g):
        big = np.abs(gW) > 1e-6
        assert np.allclose((W - W2)[big], 1e-3 * np.sign(gW[big]), rtol=1e-3)


def test_training_fits_a_smooth_function():
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (256, 8))
    T = np.stack([np.sin(2 * X[:, 0]) + X[:, 1] ** 2, X[:, 2] * X[:, 3]], axis=1)
    M = np.ones_like(T)
    params = mlp.init_params([8, 32, 32, 32, 2], 1)
    st = {}
    l0 = mlp.loss(params, X, T, M)
    for _ in range(300):
        params = mlp.adam_step(params, mlp.gradients(params, X, T, M), st, lr=3e-3)
    assert mlp.loss(params, X, T, M) < 0.05 * l0
