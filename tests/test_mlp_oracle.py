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


# ---- hand-worked example: features and bounds written out -----------------
# B (4 x 10):  row 0 = {1, 4, 7}, row 1 = {2}, row 2 = {}, row 3 = {0, 3, 5, 6, 9}
# A (4 x 4):   row 0 = {0, 1}, row 1 = {1, 2, 3}, row 2 = {2}, row 3 = {}
#   row 0: lists of 3 and 1 entries -> 2 lists, 4 products, longest 3, shortest 1,
#          columns 1..7 -> span 7
#   row 1: lists of 1, 0, 5 entries -> 3 lists, 6 products, longest 5, shortest 0,
#          columns 0..9 -> span 10
#   row 2: one empty list -> 1 list, 0 products, longest = shortest = 0, span 0
#   row 3: no list
def _hand_example():
    B = synth.CSR(4, 10, np.array([0, 3, 4, 4, 9], np.int32),
                  np.array([1, 4, 7, 2, 0, 3, 5, 6, 9], np.int32), np.ones(9))
    A = synth.CSR(4, 4, np.array([0, 2, 5, 6, 6], np.int32), np.array([0, 1, 1, 2, 3, 2], np.int32), np.ones(6))
    return A, B


def test_row_features_hand_example():
    A, B = _hand_example()
    f = oracle.row_features(A, B)
    assert list(f["nnza"]) == [2, 3, 1, 0]
    assert list(f["nprod"]) == [4, 6, 0, 0]
    assert list(f["maxb"]) == [3, 5, 0, 0]
    assert list(f["minb"]) == [1, 0, 0, 0]
    assert list(f["span"]) == [7, 10, 0, 0]


def test_raw_features_hand_example():
    A, B = _hand_example()
    f = oracle.row_features(A, B)
    x = mlp.raw_features(f["nnza"], f["nprod"], f["maxb"], f["minb"], f["span"], B.cols)
    want = np.array([
        # log1p(lists), log((1+nprod)/N), log1p(maxb), log1p(minb), log(span/N), log1p(nprod/span)
        [1.0986122886681098, -0.6931471805599453, 1.3862943611198906, 0.6931471805599453,
         -0.35667494393873245, 0.4519851237430572],   # ln 3, ln 0.5, ln 4, ln 2, ln 0.7, ln(11/7)
        [1.3862943611198906, -0.35667494393873245, 1.791759469228055, 0.0,
         0.0, 0.47000362924573563],                    # ln 4, ln 0.7, ln 6, 0, ln 1, ln 1.6
        [0.6931471805599453, -2.3025850929940455, 0.0, 0.0,
         -2.3025850929940455, 0.0],                    # ln 2, ln 0.1, 0, 0, span 0 taken as 1, 0
        [0.0, -2.3025850929940455, 0.0, 0.0, -2.3025850929940455, 0.0],
    ])
    assert np.allclose(x, want, rtol=0, atol=1e-15)


def test_forward_hand_computed():
    # one path through each layer: W1[2][5] = 0.5, b1[5] = -1; W2[5][7] = 2,
    # b2[7] = 0.25; W2[5][9] = -1, b2[9] = 0.5; W3[7] = -3, W3[9] = 10, b3 = 0.125
    p = mlp.unpack(np.zeros(mlp.N_PARAMS))
    p["W1"][2, 5] = 0.5
    p["b1"][5] = -1.0
    p["W2"][5, 7] = 2.0
    p["b2"][7] = 0.25
    p["W2"][5, 9] = -1.0
    p["b2"][9] = 0.5
    p["W3"][7] = -3.0
    p["W3"][9] = 10.0
    p["b3"][0] = 0.125
    theta = mlp.pack(p)
    assert theta[2 * 64 + 5] == 0.5  # row-major W1[6][64]: input 2 feeds hidden unit 5
    x = np.zeros((3, 6))
    x[0, 2] = 4.0   # z1 = 1 (active); z2[7] = 2.25 (active), z2[9] = -0.5 (inactive)
    x[1, 2] = 1.0   # z1 = -0.5 (inactive); z2[7] = 0.25, z2[9] = 0.5 (both active)
    x[2, 1] = 4.0   # input 1 feeds nothing
    y, _ = mlp.forward(theta, x)
    assert list(y) == [-3.0 * 2.25 + 0.125, -3.0 * 0.25 + 10.0 * 0.5 + 0.125, -3.0 * 0.25 + 10.0 * 0.5 + 0.125]
    assert list(y) == [-6.625, 4.375, 4.375]
