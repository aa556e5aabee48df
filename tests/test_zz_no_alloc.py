"""The gradient entry point that allocates nothing (its sample indices and per-wavefront
gradient partials live in a fixed device array) against ucac_mlp_grad, which allocates
the same buffers per call: the same kernels, so the gradient and the loss agree bit for
bit.  Two calls in a row, the second with a smaller input, then a size beyond the fixed
array's limit, which the call rejects before launching anything."""
import numpy as np
import pytest

from oracle import mlp as om
from paper_2310_13145_amd import ucac

pytestmark = pytest.mark.gpu


def _case(rng, n):
    X = (rng.normal(0.0, 1.0, (n, ucac.MLP_IN)) * rng.uniform(0.2, 2.0, ucac.MLP_IN)).astype(np.float32)
    Y = rng.normal(0.0, 0.5, (n, ucac.MLP_OUT)).astype(np.float32)
    return X, Y


def test_noalloc_gradient_matches_allocating_entry_point():
    import torch
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(77)
    vec = (om.init_params(5) + rng.normal(0, 0.02, ucac.MLP_PARAMS)).astype(np.float32)
    net = ucac.WarmStartNet(seed=2)
    net.set_weights(vec)
    grad = torch.empty(ucac.MLP_PARAMS, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    for n in (ucac.MLP_NOALLOC_MAX, 1000, 37):
        print(f"[noalloc] n={n}", flush=True)
        X, Y = _case(rng, n)
        g_ref, l_ref = net.grad(X, Y)
        xd, td = torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev)
        grad.fill_(np.nan)
        loss.fill_(np.nan)
        net.grad_noalloc(xd, td, grad, loss)
        torch.cuda.synchronize()
        g = grad.cpu().numpy()
        np.testing.assert_array_equal(g, g_ref)
        assert float(loss.cpu()[0]) / (4.0 * n) == l_ref
    # the weights are unchanged
    np.testing.assert_array_equal(net.get_weights(), vec)
    # beyond the fixed array's size: rejected, with the limit in the message
    X, Y = _case(rng, ucac.MLP_NOALLOC_MAX + 1)
    with pytest.raises(ucac.UcacError) as e:
        net.grad_noalloc(torch.from_numpy(X).to(dev), torch.from_numpy(Y).to(dev), grad, loss)
    assert e.value.code == ucac.UCAC_E_INVAL and str(ucac.MLP_NOALLOC_MAX) in str(e.value)
    net.close()
