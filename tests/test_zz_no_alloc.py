"""The gradient entry point that allocates nothing (static workspace) against
cphot_surrogate_gradient, through the C ABI: equal results bit for bit on two
calls in a row, the second with a smaller batch; sizes beyond the workspace are
rejected."""
import math

import numpy as np
import pytest

from paper_2405_04229_amd import cphot
from paper_2405_04229_amd import workload as W

pytestmark = pytest.mark.gpu


def _inputs(torch, n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = np.array(W.SURROGATE_LO), np.array(W.SURROGATE_HI)
    X = lo + (hi - lo) * rng.random((n, 5))
    Y = rng.normal(0.0, 1.0, (n, 4)) * np.array([3.0, 0.5, 0.2, 0.1]) + np.array([1.0, 0.0, 0.3, -0.2])
    return (torch.from_numpy(X.astype(np.float32)).cuda(), torch.from_numpy(Y.astype(np.float32)).cuda())


def test_gradient_without_allocation_equals_gradient():
    import torch
    sur = cphot.Surrogate(W.SURROGATE_LO, W.SURROGATE_HI, max_batch=8192, init_seed=3)
    rng = np.random.default_rng(11)
    th = rng.normal(0.0, 0.2, cphot.N_PARAMS).astype(np.float32)
    lo, hi = np.array(W.SURROGATE_LO), np.array(W.SURROGATE_HI)
    norm = np.zeros(cphot.N_NORM, dtype=np.float32)
    norm[0:5], norm[5:10], norm[10:15] = lo, hi, 2.0 / (hi - lo)
    norm[16:20], norm[20:24] = [1.0, 0.0, 0.3, -0.2], [3.0, 0.5, 0.2, 0.1]
    sur.set_params(th, norm)
    grad = torch.full((cphot.N_PARAMS,), math.nan, dtype=torch.float32, device="cuda")
    loss = torch.full((1,), math.nan, dtype=torch.float32, device="cuda")
    for n, seed in ((4096, 1), (1024, 2)):
        print(f"no-alloc gradient: n={n} seed={seed}", flush=True)
        X, Y = _inputs(torch, n, seed)
        g_ref, l_ref = sur.gradient(X, Y)
        sur.gradient_noalloc(X, Y, grad, loss)
        torch.cuda.synchronize()
        assert torch.isfinite(g_ref).all() and float(g_ref.abs().sum()) > 0
        assert torch.equal(grad, g_ref), float((grad - g_ref).abs().max())
        assert torch.equal(loss, l_ref)
    # beyond the static workspace: rejected before anything is enqueued
    X, Y = _inputs(torch, 8192, 3)
    with pytest.raises(cphot.CphotError, match="4096"):
        sur.gradient_noalloc(X, Y, grad, loss)
    with pytest.raises(cphot.CphotError):
        sur.gradient_noalloc(X[:100], Y[:100], grad, loss)
    sur.close()
