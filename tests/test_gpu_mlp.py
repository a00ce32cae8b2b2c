"""Skip-network kernels (forward, gradient, Adam training) on the GPU against
the FP64 CPU reference (oracle/mlp_ref.py, itself pinned by finite
differences).  The GPU computes in FP32: tolerances are FP32-level."""
import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_2009_03551_amd import tc2 as T

pytestmark = pytest.mark.gpu


def problem(n=3000, seed=0):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.2, M.NPARAM).astype(np.float32)
    X = rng.normal(0, 1, (n, M.NF)).astype(np.float32)
    y = (rng.random(n) > 0.4).astype(np.float32)
    return theta, X, y


def test_forward_matches_reference():
    theta, X, _ = problem()
    z = T.mlp_forward(theta, X)
    zr = M.forward(theta.astype(np.float64), X.astype(np.float64))
    np.testing.assert_allclose(z, zr, rtol=1e-4, atol=1e-5 * np.abs(zr).max())


def test_gradient_matches_reference():
    theta, X, y = problem()
    g, loss = T.mlp_grad(theta, X, y)
    lr, gr = M.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    assert abs(loss - lr) < 1e-5 * abs(lr)
    err = np.abs(g - gr).max() / np.abs(gr).max()
    print(f"  max grad error relative to max |grad|: {err:.2e}")
    assert err < 1e-4


def test_one_adam_step_matches_reference():
    theta, X, y = problem(n=1000, seed=3)
    th1, losses = T.mlp_train(X, y, theta, epochs=1, batch=1000, lr=1e-2)
    _, gr = M.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), y.astype(np.float64))
    ref, _, _ = M.adam_step(theta.astype(np.float64), np.zeros(M.NPARAM), np.zeros(M.NPARAM), gr, 1,
                            lr=1e-2)
    # where the gradient is not tiny, the first Adam step moves by lr * sign(g)
    big = np.abs(gr) > 1e-4 * np.abs(gr).max()
    np.testing.assert_allclose(th1[big], ref[big], atol=2e-5)


def test_training_reduces_loss_on_separable_data():
    rng = np.random.default_rng(5)
    X = rng.normal(0, 1, (20000, M.NF)).astype(np.float32)
    y = ((X[:, 0] - 0.5 * X[:, 3] + 0.25 * X[:, 5] ** 2) > 0.2).astype(np.float32)
    theta0 = (rng.normal(0, 1, M.NPARAM) * 0.1).astype(np.float32)
    th, losses = T.mlp_train(X, y, theta0, epochs=15, batch=512, lr=3e-3)
    print(f"  loss per epoch: {losses[0]:.4f} -> {losses[-1]:.4f}")
    assert losses[-1] < 0.5 * losses[0]
    acc = np.mean((T.mlp_forward(th, X) > 0) == (y > 0.5))
    assert acc > 0.95


def test_rejects_bad_input():
    theta, X, y = problem(n=10)
    X[0, 0] = np.nan
    with pytest.raises(T.TC2Error):
        T.mlp_grad(theta, X, y)
