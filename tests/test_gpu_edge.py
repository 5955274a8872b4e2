"""Edge and degenerate cases of the GPU path: special physics with closed forms, grids
that multigrid cannot coarsen, tiny grids, bad inputs and error codes."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_1904_00182_amd import nc, inputs, workloads
from gpu_helpers import oracle_params, oracle_blob_design, check_fields, to_dev, DEV

pytestmark = pytest.mark.gpu


def _solve(p, x):
    sol = nc.Solver(p, DEV)
    sol.set_design(to_dev(x))
    s = sol.solve_state()
    assert sol.last_info["status"] == nc.NC_OK, sol.last_info
    return sol, s


def test_conduction_limit_adjoint_equals_temperature():
    """Gr = 0: P = u = 0, lambda_T = t and the sensitivity is non-positive."""
    p = workloads.problem((16, 8, 16), 1e3, alpha=0.0)
    x = inputs.noise_design(16 * 8 * 16, 2)
    sol, s = _solve(p, x)
    lam = sol.solve_adjoint(s, sol.objective_grad())
    sn, ln = s.cpu().numpy(), lam.cpu().numpy()
    assert np.abs(sn[:, 3]).max() < 1e-14 and np.abs(sn[:, :3]).max() < 1e-14
    assert np.linalg.norm(ln[:, 4] - sn[:, 4]) / np.linalg.norm(sn[:, 4]) < 1e-10
    assert (sol.sensitivity(s, lam).cpu().numpy() <= 1e-18).all()


def test_zero_flux_gives_zero_solution():
    p = workloads.problem((8, 4, 8), 1e3, q_h=0.0)
    sol, s = _solve(p, inputs.noise_design(256, 1))
    assert float(s.abs().max()) == 0.0
    lam = sol.solve_adjoint(s, sol.objective_grad())
    assert float(lam.abs().max()) == 0.0


@pytest.mark.parametrize("grid", [(1, 1, 1), (2, 2, 2), (9, 5, 7), (21, 11, 9)])
def test_uncoarsenable_and_tiny_grids_match_oracle(grid):
    """Odd sizes (one multigrid level: a dense direct coarse solve, or block-Jacobi
    smoothing only when the dense matrix would be too large) and one-element grids."""
    p = workloads.problem(grid, 1e4, q_h=3.0)
    E = grid[0] * grid[1] * grid[2]
    x = inputs.noise_design(E, 6)
    sol, s = _solve(p, x)
    m = oracle.Model(oracle_params(p), x)
    so, _ = m.solve_state()
    check_fields(s.cpu().numpy(), so, 1e-8, f"state {grid}")


@pytest.mark.parametrize("fill", [0.0, 1.0])
def test_uniform_designs(fill):
    """All fluid (strongest convection) and all solid (conduction, kappa_s)."""
    p = workloads.problem((16, 8, 16), 1e4, q_h=2.0)
    x = np.full(16 * 8 * 16, fill)
    sol, s = _solve(p, x)
    m = oracle.Model(oracle_params(p), x)
    so, _ = m.solve_state()
    check_fields(s.cpu().numpy(), so, 1e-8, f"state fill {fill}")


def test_blob_designs_are_bit_identical_to_oracle_recipe():
    """The thresholded cone-filtered designs built by the GPU filter and by the oracle's
    filter are the same 0/1 fields (64x32x64 seed 1, 32x16x32 seed 1)."""
    for grid, seed in (((64, 32, 64), 1), ((32, 16, 32), 1), ((128, 64, 128), 2)):
        xg = workloads.design(grid, "blobs", seed, DEV).cpu().numpy()
        xo = oracle_blob_design(grid, seed)
        assert np.array_equal(xg, xo)
        assert 0.2 < xg.mean() < 0.8


def test_cavity32_blobs_state_and_adjoint_vs_oracle():
    """The oracle-size member of the 64x32x64 workload family (32x16x32, seed 1): float64
    multigrid-FGMRES state and adjoint within 1e-8 of SuperLU."""
    p, x, cfg = workloads.config("cavity32", DEV)
    sol = nc.Solver(p, DEV)
    sol.set_design(x)
    s = sol.solve_state()
    lam = sol.solve_adjoint(s, sol.objective_grad())
    dfdx = sol.sensitivity(s, lam).cpu().numpy()
    m = oracle.Model(oracle_params(p), x.cpu().numpy())
    so, _ = m.solve_state()
    lo = m.solve_adjoint(so, m.dfds())
    _, go = m.sensitivity(so, lo)
    check_fields(s.cpu().numpy(), so, 1e-8, "state")
    check_fields(lam.cpu().numpy(), lo, 1e-8, "adjoint")
    check_fields(dfdx, go, 1e-8, "dfdx")


def test_error_codes():
    lib = nc.load()
    p = workloads.problem((8, 4, 8), 1e3)
    need = nc.workspace_bytes(p)
    ws = torch.empty(need // 2, dtype=torch.uint8, device=DEV)
    ctx = ctypes.c_void_p()
    assert lib.nc_create(ctypes.byref(p), ctypes.c_void_p(ws.data_ptr()), need // 2, None, ctypes.byref(ctx)) == nc.NC_ENOMEM
    sol = nc.Solver(p, DEV)
    x = torch.full((sol.E,), 0.5, dtype=torch.float64, device=DEV)
    x[3] = float("nan")
    sol.set_design(x)
    with pytest.raises(nc.NCError) as ei:
        sol.solve_state()
    assert ei.value.status == nc.NC_ENAN
    bad = nc.default_problem(8, 4, 8, krylov_restart=40)
    assert nc.workspace_bytes(bad) == 0
    # solving before a design is set is rejected
    sol2 = nc.Solver(p, DEV)
    with pytest.raises(nc.NCError) as ei:
        sol2.solve_state()
    assert ei.value.status == nc.NC_EINVAL
