"""tc2_mlp_grad_noalloc (the gradient of the skip network for callers that
cannot allocate) against tc2_mlp_grad on the same inputs, through the C ABI:
two calls in a row, the second with fewer samples, then a call at the size
limit, and the limit itself.  Both entry points run the same gradient and
summation kernels; the per-block sums use float atomics in LDS, whose order
can vary, so the bar is FP32-level (as the gradient's own parity test)."""
import numpy as np
import pytest
import torch

from paper_2009_03551_amd import tc2 as T

pytestmark = pytest.mark.gpu


def problem(n, seed):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.2, T.MLP_PARAMS).astype(np.float32)
    X = rng.normal(0, 1, (n, T.MLP_IN)).astype(np.float32)
    y = (rng.random(n) > 0.4).astype(np.float32)
    return theta, X, y


def noalloc(theta, X, y):
    dev = torch.device("cuda:0")
    th, xx, yy = (torch.from_numpy(a).to(dev) for a in (theta, X, y))
    g = torch.full((T.MLP_PARAMS,), float("nan"), dtype=torch.float32, device=dev)
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    T.mlp_grad_noalloc(th.data_ptr(), xx.data_ptr(), yy.data_ptr(), len(y), g.data_ptr(),
                       loss.data_ptr(), stream=stream)
    torch.cuda.synchronize()
    return g.cpu().numpy(), float(loss.cpu()[0])


def check(theta, X, y):
    g, loss = noalloc(theta, X, y)
    gr, lr = T.mlp_grad(theta, X, y)
    err = np.abs(g - gr).max() / np.abs(gr).max()
    print(f"  n={len(y)}: loss {loss:.8f} vs {lr:.8f}, grad error {err:.2e}", flush=True)
    assert abs(loss - lr) <= 1e-6 * abs(lr)
    assert err < 1e-5


def test_noalloc_gradient_equals_the_allocating_one():
    check(*problem(9000, 1))
    check(*problem(700, 2))          # a second, smaller call on the same scratch
    check(*problem(T.MLP_NOALLOC_MAX_N, 3))


def test_noalloc_rejects_sizes_beyond_its_scratch():
    theta, X, y = problem(8, 4)
    with pytest.raises(T.TC2Error):
        T.mlp_grad_noalloc(1, 1, 1, T.MLP_NOALLOC_MAX_N + 1, 1, 1)
    with pytest.raises(T.TC2Error):
        T.mlp_grad_noalloc(1, 1, 1, 0, 1, 1)
