"""The allocation-free dense inverse (nc_dense_inverse_noalloc, static per-GPU scratch)
against nc_dense_inverse with caller-provided scratch: two calls in a row, the second on
a smaller matrix, each bitwise equal to the workspace variant (the same kernels run on
the same input) and a true inverse."""

import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _matrix(n, seed):
    r = np.random.default_rng(seed)
    a = r.standard_normal((n, n)) + n ** 0.5 * np.eye(n)
    a[np.arange(n), np.arange(n)] *= r.choice([0.0, 1.0], n)       # zero diagonals force pivoting
    return a


@pytest.mark.parametrize("sizes", [(400, 240), (150, 37)])
def test_noalloc_matches_workspace_variant(sizes):
    import torch
    from paper_1904_00182_amd import nc
    dev = "cuda:0"
    for k, n in enumerate(sizes):
        print(f"noalloc dense inverse: call {k}, n={n}", flush=True)
        a = _matrix(n, 10 * n + k)
        ref_inv, ref_tr = nc.dense_inverse(torch.as_tensor(a, device=dev))
        buf = torch.zeros(2 * n * n, dtype=torch.float64, device=dev)
        buf[: n * n].copy_(torch.as_tensor(a.ravel(), device=dev))
        before = torch.cuda.memory_allocated(dev)
        nc.dense_inverse_noalloc(buf, n)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated(dev) == before
        inv = buf[: n * n].view(n, n)
        tr = buf[n * n:].view(n, n)
        assert torch.equal(inv, ref_inv) and torch.equal(tr, ref_tr)
        x = inv.cpu().numpy()
        assert np.abs(a @ x - np.eye(n)).max() < 1e-9 * np.linalg.cond(a)
        assert np.array_equal(tr.cpu().numpy(), x.T)
