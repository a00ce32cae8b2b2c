"""Learned block skip: logged training data, GPU-trained network, and what it
gains over the exact norm-bound screen on a system it was not trained on.
The error the network introduces is measured against the exact-screen solve."""
import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_2009_03551_amd import skipnet
from paper_2009_03551_amd import tc2 as T
from paper_2009_03551_amd import workloads as W

pytestmark = pytest.mark.gpu


def dense_x1(r):
    return [T.bsr_dense(x) for x in r.X1]


@pytest.fixture(scope="module")
def trained():
    train_sys = [W.config_system("cube10", L=L, seed=500 + L, eps=1e-5) for L in (5, 6, 7)]
    x, y = skipnet.collect(train_sys)
    print(f"  logged {len(y)} candidates, dropped fraction {y.mean():.3f}", flush=True)
    theta, losses = skipnet.train(x, y, epochs=25)
    print(f"  training loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    return theta, losses, x, y


def test_logged_features_are_finite_and_labelled(trained):
    _, _, x, y = trained
    assert len(y) > 1000
    assert np.all(np.isfinite(x))
    assert set(np.unique(y)) <= {0.0, 1.0}
    assert 0.02 < y.mean() < 0.98


def test_training_reduces_loss(trained):
    _, losses, _, _ = trained
    assert losses[-1] < 0.7 * losses[0]


def test_network_gain_over_exact_screen(trained):
    theta = trained[0]
    s = W.config_system("cube10", L=7, seed=42, eps=1e-5)      # not a training system
    a = T.solve(s, skip="bound", profile=True)[0]
    b = T.solve(s, skip="mlp", mlp_weights=theta, mlp_threshold=0.995, profile=True)[0]
    dx1 = max(np.abs(p - q).max() for p, q in zip(dense_x1(a), dense_x1(b)))
    dal = abs(a.alpha[0] - b.alpha[0]) / abs(a.alpha[0])
    gain = 1.0 - b.executed_flops / a.executed_flops
    print(f"  exact screen: {a.screened_blocks} skipped, {a.executed_flops / 1e12:.3f} TF; "
          f"network: +{b.mlp_skipped_blocks} skipped, {b.executed_flops / 1e12:.3f} TF "
          f"({100 * gain:.1f}% less); max|dX1| vs exact screen {dx1:.2e}, rel|dalpha| {dal:.2e}",
          flush=True)
    assert b.mlp_skipped_blocks > 0 and b.mlp_updates > 0
    assert b.executed_flops < a.executed_flops
    # every output the network skipped had an exact bound below 4 eps (the
    # default cap): the error it injects per block is below that
    assert dx1 < 4 * s.eps


def test_network_budget_falls_back_to_the_exact_screen(trained):
    # a budget on the summed bounds of the skipped outputs: once it is spent,
    # the rest of the solve runs with the exact screen; the result meets the
    # 1e-6 gate against the exact-screen solve
    theta = trained[0]
    s = W.config_system("cube10", L=7, seed=42, eps=1e-5)
    a = T.solve(s, skip="bound")[0]
    b = T.solve(s, skip="mlp", mlp_weights=theta, mlp_threshold=0.995, mlp_budget=1e-6)[0]
    dx1 = max(np.abs(p - q).max() for p, q in zip(dense_x1(a), dense_x1(b)))
    dal = abs(a.alpha[0] - b.alpha[0]) / abs(a.alpha[0])
    print(f"  network ran {b.mlp_updates} of {b.iters} updates, skipped {b.mlp_skipped_blocks}; "
          f"max|dX1| {dx1:.2e}, rel|dalpha| {dal:.2e}", flush=True)
    assert b.mlp_updates < b.iters
    assert dx1 < 1e-6 and dal < 1e-6


def test_in_kernel_logits_match_the_reference_forward(trained):
    # the network evaluated inside the numeric kernel (one hidden unit per
    # lane, W2 transposed in LDS) against the FP64 reference forward on the
    # same logged features; the logged skip decisions follow the logits
    theta = trained[0]
    s = W.config_system("cube10", L=5, seed=77, eps=1e-5)
    thr = 0.9
    sv = T.Solver(s, skip="mlp", mlp_weights=theta, mlp_threshold=thr, log_capacity=2_000_000,
                  export=False)
    try:
        r = sv.run()[0]
        x, y, z = sv.log(logits=True)
    finally:
        sv.close()
    zr = M.forward(theta.astype(np.float64), x.astype(np.float64))
    err = np.abs(z - zr).max() / max(1.0, np.abs(zr).max())
    print(f"  {len(z)} logged candidates, {int((y < 0).sum())} skipped by the network; "
          f"max |logit - reference| / max(1, max |logit|) = {err:.2e}", flush=True)
    assert len(z) > 1000 and (y < 0).sum() > 0 and r.mlp_skipped_blocks == (y < 0).sum()
    assert err < 1e-4
    zt = np.log(thr / (1 - thr))
    assert np.all(z[y < 0] > zt)          # every skipped candidate passed the threshold
