"""Pins of the CPU reference of the size predictor: central finite
differences for the gradient, a closed form of Adam's first step, a network
with zero hidden weights, and the size bounds of the features."""
import numpy as np
import pytest

import oracle
import synth
from oracle import mlp


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    theta = mlp.init_params(seed).astype(np.float64)
    theta += rng.standard_normal(theta.size) * 0.01  # non-zero biases too
    x = rng.standard_normal((7, 6))
    t = rng.standard_normal(7)
    _, g = mlp.loss_and_grad(theta, x, t)
    idx = rng.choice(theta.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(theta)
        e[i] = h
        lp, _ = mlp.loss_and_grad(theta + e, x, t)
        lm, _ = mlp.loss_and_grad(theta - e, x, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd))


def test_zero_hidden_network_is_its_output_bias():
    theta = np.zeros(mlp.N_PARAMS)
    p = mlp.unpack(theta)
    p["b3"][0] = 0.75
    theta = mlp.pack(p)
    x = np.random.default_rng(1).standard_normal((5, 6))
    y, _ = mlp.forward(theta, x)
    assert np.all(y == 0.75)
    t = np.arange(5.0)
    loss, g = mlp.loss_and_grad(theta, x, t)
    assert loss == pytest.approx(np.mean((0.75 - t) ** 2))
    gp = mlp.unpack(g)
    assert gp["b3"][0] == pytest.approx(2 * np.mean(0.75 - t))
    assert np.all(g[:-1] == 0)  # no signal reaches the dead ReLU layers


def test_adam_first_step_closed_form():
    # with m = v = 0 the first step moves every weight by lr * g / (|g| + eps)
    g = np.array([3.0, -2e-3, 0.0, 5e-9])
    theta = np.ones(4)
    new, m, v = mlp.adam_step(theta, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    assert np.allclose(new, 1.0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_converges_on_quadratic():
    theta = np.array([5.0, -3.0])
    m = v = np.zeros(2)
    for t in range(1, 3001):
        theta, m, v = mlp.adam_step(theta, 2 * theta, m, v, t, lr=0.05)
    assert np.all(np.abs(theta) < 1e-3)


def test_parameter_count():
    assert mlp.N_PARAMS == 6 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4673


def test_feature_bounds_hold():
    A = synth.rmat(10, 8, 4)
    f = oracle.row_features(A, A)
    r = oracle.spgemm(A, A)
    nnzc = np.diff(r.rpt)
    ok = f["nprod"] > 0
    assert np.all(nnzc[ok] >= f["maxb"][ok]) and np.all(nnzc[ok] <= np.minimum(f["nprod"], f["span"])[ok])
    single = f["nnza"] == 1
    assert np.all(nnzc[single] == f["nprod"][single])
    x = mlp.raw_features(f["nnza"], f["nprod"], f["maxb"], f["minb"], f["span"], A.cols)
    assert x.shape == (A.rows, 6) and np.all(np.isfinite(x))


def test_predict_sizes_clamps():
    s = mlp.predict_sizes(np.array([0.0, -50.0, 3.0]), 0.0, np.array([10, 10, 10]), np.array([2, 4, 1]),
                          np.array([10, 8, 7]))
    assert list(s) == [10, 4, 7]
