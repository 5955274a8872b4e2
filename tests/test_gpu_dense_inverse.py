"""The multigrid's coarsest-grid inverse (nc_dense_inverse) against LAPACK's through
numpy, on seeded matrices: both the single-workgroup register path (n <= 160) and the
multi-workgroup path, pivoting forced by a zero diagonal, and the stored transpose."""

import numpy as np
import pytest
import torch

from paper_1904_00182_amd import nc
from gpu_helpers import DEV

pytestmark = pytest.mark.gpu


def _matrix(n, seed, zero_diag):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n)) + 2.0 * np.sqrt(n) * np.eye(n)[rng.permutation(n)]
    if zero_diag and n > 1:
        a[np.arange(n), np.arange(n)] = 0.0   # no step can pivot in place
    return a


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 129, 150, 160, 161, 300, 1000])
@pytest.mark.parametrize("zero_diag", [False, True], ids=["dense", "zero_diag"])
def test_dense_inverse_matches_lapack(n, zero_diag):
    a = _matrix(n, 1000 + n, zero_diag)
    inv, inv_t = nc.dense_inverse(torch.as_tensor(a, device=DEV))
    torch.cuda.synchronize()
    got, got_t = inv.cpu().numpy(), inv_t.cpu().numpy()
    ref = np.linalg.inv(a)
    # forward error within a small multiple of cond(A) * n * eps
    bound = 50.0 * n * np.finfo(np.float64).eps * np.linalg.cond(a)
    assert np.abs(got - ref).max() <= bound * np.abs(ref).max(), (np.abs(got - ref).max(), bound)
    assert np.abs(got @ a - np.eye(n)).max() <= bound
    assert np.array_equal(got_t, got.T)


def test_dense_inverse_largest_size_and_repeat():
    """n = NC_DENSE_MAX, then a smaller matrix through the same call: results do not
    depend on earlier calls."""
    for n in (nc.NC_DENSE_MAX, 150):
        a = _matrix(n, 7, True)
        inv, _ = nc.dense_inverse(torch.as_tensor(a, device=DEV))
        got = inv.cpu().numpy()
        ref = np.linalg.inv(a)
        bound = 50.0 * n * np.finfo(np.float64).eps * np.linalg.cond(a)
        assert np.abs(got - ref).max() <= bound * np.abs(ref).max()


def test_dense_inverse_is_deterministic():
    a = torch.as_tensor(_matrix(150, 3, True), device=DEV)
    x1, _ = nc.dense_inverse(a)
    x2, _ = nc.dense_inverse(a)
    assert torch.equal(x1, x2)
