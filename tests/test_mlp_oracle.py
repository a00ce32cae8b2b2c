"""Pins of the FP64 MLP reference: finite differences, hand-computed cases."""
import numpy as np

from oracle import mlp_ref as M


def rand_problem(n=7, seed=0):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.3, M.NPARAM)
    X = rng.normal(0, 1, (n, M.NF))
    y = (rng.random(n) > 0.5).astype(float)
    return theta, X, y


def test_param_count():
    assert M.NPARAM == 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1 == 4801


def test_gradient_matches_central_differences():
    theta, X, y = rand_problem()
    _, g = M.loss_and_grad(theta, X, y)
    rng = np.random.default_rng(1)
    idx = rng.choice(M.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [M.NPARAM - 1, 0, 64 * 8 + 3]])   # b3, W1[0,0], b1[3]
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.loss_and_grad(tp, X, y)[0] - M.loss_and_grad(tm, X, y)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_weights_hand_case():
    # all weights zero: z = b3 for every sample, loss = softplus(b3) - mean(y) b3
    theta = np.zeros(M.NPARAM)
    theta[-1] = 0.5
    X = np.ones((4, M.NF))
    y = np.array([1.0, 0.0, 1.0, 1.0])
    loss, g = M.loss_and_grad(theta, X, y)
    assert abs(loss - (np.log1p(np.exp(0.5)) - 0.75 * 0.5)) < 1e-15
    sig = 1.0 / (1.0 + np.exp(-0.5))
    assert abs(g[-1] - (sig - 0.75)) < 1e-15
    assert not np.any(g[:-1])          # ReLU of zero: no gradient reaches the rest


def test_single_path_hand_case():
    # one active path: x0 -> h1_0 -> h2_0 -> z with weights 2, 3, 4
    theta = np.zeros(M.NPARAM)
    p = M.unpack(theta)             # views into theta
    p["W1"][0, 0] = 2.0
    p["W2"][0, 0] = 3.0
    p["w3"][0] = 4.0
    X = np.zeros((1, M.NF))
    X[0, 0] = 0.25
    assert M.forward(theta, X)[0] == 4.0 * 3.0 * 2.0 * 0.25
    _, g = M.loss_and_grad(theta, X, np.array([0.0]))
    dz = 1.0 / (1.0 + np.exp(-6.0))
    assert abs(g[0] - dz * 4.0 * 3.0 * 0.25) < 1e-14          # dW1[0,0]
    assert abs(g[64 * 8 + 64] - dz * 4.0 * 2.0 * 0.25) < 1e-14  # dW2[0,0]


def test_adam_hand_step():
    theta = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    t1, m, v = M.adam_step(theta, np.zeros(2), np.zeros(2), g, 1, lr=0.1)
    # first step: m_hat = g, v_hat = g^2  ->  theta - lr * sign(g) (up to eps)
    np.testing.assert_allclose(t1, [0.9, -1.9], atol=1e-7)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
