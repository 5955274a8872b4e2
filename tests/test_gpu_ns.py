"""Parity of the GPU Navier-Stokes / Brinkman solver (nc_ns_* entry points) with the
oracle's model: residual and Jacobian rows element by element, Newton state, adjoint,
objective and sensitivities on the cavity and on the quarter benchmark with symmetry
planes, heat-source block, passive regions and the PDE filter; preconditioner pairing
and bitwise reproducibility."""

import numpy as np
import pytest
import torch

import oracle
from paper_1904_00182_amd import nc, inputs

from gpu_helpers import DEV, oracle_params, random_state, check_fields, to_dev

pytestmark = pytest.mark.gpu


def _quarter_kw(n):
    """Quarter cavity of Sec. 6.1 on an n x n x 2n grid of edge 1/(2n): source block on the
    floor (solid), design box inside, symmetry planes x = y = 1/2."""
    L = 1.0
    src = (0.375 * L, 0.5 * L, 0.375 * L, 0.5 * L, 0.0, 0.125 * L)
    des = (0.125 * L, 0.5 * L, 0.125 * L, 0.5 * L, 0.125 * L, 0.875 * L)
    return dict(h=1.0 / (2 * n), q_h=0.0, Q=40.0, q_box=src, solid_box=src, design_box=des, sym_x=1, sym_y=1)


CASES = {
    "cavity8": ((8, 4, 8), dict(alpha=1e3, q_h=5.0)),
    "ragged7x5x6": ((7, 5, 6), dict(alpha=1e3, q_h=5.0, Q=20.0, q_box=(0.3, 0.7, 0.2, 0.8, 0.0, 0.4))),
    "quarter4": ((4, 4, 8), dict(alpha=1e3, **_quarter_kw(4))),
}


# the adjoint's residual is that of the equilibrated system; its continuity rows leave the
# adjoint pressure about 100x the residual, hence a tighter target than the Darcy model's
ADJ_RTOL = 1e-12


def _pair(grid, kw, seed, precision=nc.NC_FP64, **extra):
    p = nc.default_problem(*grid, precision=precision, adjoint_rtol=ADJ_RTOL, kappa_s=1e5, smooth_omega=0.7, **kw,
                           **extra)
    x = inputs.noise_design(grid[0] * grid[1] * grid[2], seed)
    model = oracle.NSModel(oracle_params(p), x)
    sol = nc.NSSolver(p, DEV)
    sol.set_design(to_dev(x))
    return p, x, model, sol


def _rows_close(a, b, tol, what):
    a = np.asarray(a)
    b = np.asarray(b)
    for f in range(5):
        scale = np.abs(b[:, f]).max()
        err = np.abs(a[:, f] - b[:, f]).max()
        assert err <= tol * max(scale, 1e-300), (what, f, err, scale)


@pytest.mark.parametrize("case", list(CASES))
def test_residual_matches_oracle(case):
    grid, kw = CASES[case]
    print("case", case, flush=True)
    p, x, model, sol = _pair(grid, kw, 3)
    s = random_state(model, 4, pscale=5.0, scale=0.05)
    r = sol.residual(to_dev(s)).cpu().numpy()
    _rows_close(r, model.residual(s), 1e-12, case)
    g = sol.gamma().cpu().numpy()
    assert np.abs(g - model.gamma).max() <= 1e-14


@pytest.mark.parametrize("case", list(CASES))
def test_jacobian_and_transpose_match_oracle(case):
    """J~ v and J~^T w of the assembled float64 Jacobian (forward-mode columns, colour-
    ordered assembly, constraints) against the oracle's complex-step Jacobian."""
    grid, kw = CASES[case]
    print("case", case, flush=True)
    p, x, model, sol = _pair(grid, kw, 5)
    s = random_state(model, 6, pscale=5.0, scale=0.05)
    J = model.jacobian(s)
    rng = inputs.rng(7)
    v = rng.standard_normal((model.mesh.n_nodes, 5))
    w = rng.standard_normal((model.mesh.n_nodes, 5))
    sol.linearize(to_dev(s))
    y = sol.jac_apply(to_dev(v)).cpu().numpy()
    yt = sol.jac_apply(to_dev(w), transpose=True).cpu().numpy()
    _rows_close(y, (J @ v.reshape(-1)).reshape(-1, 5), 1e-12, case + " J v")
    _rows_close(yt, (J.T @ w.reshape(-1)).reshape(-1, 5), 1e-12, case + " J^T w")


@pytest.mark.parametrize("precision", [nc.NC_FP64, nc.NC_MIXED])
def test_state_adjoint_sensitivity_match_oracle(precision):
    """16x8x16 cavity at Gr 1e3 with the patch flux and a volumetric source block (whose
    load weight depends on the velocity unknowns), cone filter R = 1.5: Newton state,
    compliance, d f / d s, adjoint and d f / d x against the oracle (float64 Krylov solves;
    NC_MIXED only changes the preconditioner's precision)."""
    grid = (16, 8, 16)
    kw = dict(alpha=1e3, q_h=5.0, Q=20.0, q_box=(0.375, 0.625, 0.25, 0.75, 0.0, 0.25), filter_radius=1.5)
    print("precision", precision, flush=True)
    p, x, model, sol = _pair(grid, kw, 11, precision=precision)
    s = sol.solve_state()
    info = sol.last_info
    assert info["status"] == nc.NC_OK, info
    so, ho = model.solve_state()
    assert ho["converged"]
    check_fields(s.cpu().numpy(), so, 1e-9, "ns state")
    f = sol.objective(s)
    fo = model.objective(so)
    assert abs(f - fo) <= 1e-10 * abs(fo)
    g = sol.objective_grad(s)
    go = model.dfds(so)
    check_fields(g.cpu().numpy(), go, 1e-9, "ns dfds")
    lam = sol.solve_adjoint(s, g)
    assert sol.last_info["status"] == nc.NC_OK, sol.last_info
    print("ns adjoint krylov", sol.last_info["krylov_its"], "relres", sol.last_info["rel_res"], flush=True)
    lo = model.solve_adjoint(so, go)
    check_fields(lam.cpu().numpy(), lo, 1e-8, "ns adjoint")
    dfdx = sol.sensitivity(s, lam).cpu().numpy()
    _, do = model.sensitivity(so, lo, explicit=True)
    err = np.linalg.norm(dfdx - do) / np.linalg.norm(do)
    assert err <= 1e-8 and np.abs(dfdx - do).max() <= 1e-8 * np.abs(do).max(), err
    print("ns newton", info["newton_its"], "krylov", info["krylov_its"], "levels", info["levels"], flush=True)


def test_quarter_benchmark_matches_oracle():
    """The quarter cavity of Sec. 6.1 (symmetry planes, solid heat-source block, passive
    fluid outside the design box) with the PDE filter R = 2.5: state, adjoint and
    sensitivities against the oracle."""
    grid = (8, 8, 16)
    kw = dict(alpha=1e3, filter_radius=2.5, filter_kind=nc.NC_FILTER_PDE, **_quarter_kw(8))
    p, x, model, sol = _pair(grid, kw, 13)
    s = sol.solve_state()
    assert sol.last_info["status"] == nc.NC_OK, sol.last_info
    so, _ = model.solve_state()
    check_fields(s.cpu().numpy(), so, 1e-9, "quarter state")
    g = sol.objective_grad(s)
    lam = sol.solve_adjoint(s, g)
    lo = model.solve_adjoint(so, model.dfds(so))
    check_fields(lam.cpu().numpy(), lo, 1e-8, "quarter adjoint")
    dfdx = sol.sensitivity(s, lam).cpu().numpy()
    _, do = model.sensitivity(so, lo, explicit=True)
    assert np.all(dfdx[~model.design] == 0.0)
    err = np.linalg.norm(dfdx - do) / np.linalg.norm(do)
    assert err <= 1e-8, err
    assert abs(sol.objective(s) - model.objective(so)) <= 1e-10 * abs(model.objective(so))


def test_preconditioner_transpose_pairing_and_reproducibility():
    """With as many post- as pre-sweeps on every level the V-cycle of A^T is the transpose
    of the V-cycle of A: <u, M^-1 v> = <M^-T u, v>.  Two solves give identical bits."""
    grid = (16, 8, 16)
    kw = dict(alpha=1e3, q_h=5.0)
    p, x, model, sol = _pair(grid, kw, 17)
    s = random_state(model, 18, pscale=5.0, scale=0.05)
    sol.linearize(to_dev(s))
    rng = inputs.rng(19)
    u = to_dev(rng.standard_normal((model.mesh.n_nodes, 5)))
    v = to_dev(rng.standard_normal((model.mesh.n_nodes, 5)))
    a = float((u * sol.precondition(v)).sum())
    b = float((sol.precondition(u, transpose=True) * v).sum())
    assert abs(a - b) <= 1e-10 * abs(a), (a, b)
    s1 = sol.solve_state()
    s2 = sol.solve_state()
    assert torch.equal(s1, s2)


def test_odd_grid_single_level_without_dense_coarsest():
    """9x5x9 (odd, so no coarser level; 3,000 unknowns, above the dense limit): the
    preconditioner is the smoother alone on that one level; state, adjoint and
    sensitivities still match the oracle."""
    grid = (9, 5, 9)
    kw = dict(alpha=1e3, q_h=5.0, Q=20.0, q_box=(0.3, 0.7, 0.2, 0.8, 0.0, 0.4), krylov_maxit=2000)
    p, x, model, sol = _pair(grid, kw, 23)
    s = sol.solve_state()
    info = sol.last_info
    assert info["status"] == nc.NC_OK and info["levels"] == 1, info
    so, _ = model.solve_state()
    check_fields(s.cpu().numpy(), so, 1e-9, "odd-grid state")
    g = sol.objective_grad(s)
    lam = sol.solve_adjoint(s, g)
    assert sol.last_info["status"] == nc.NC_OK, sol.last_info
    lo = model.solve_adjoint(so, model.dfds(so))
    check_fields(lam.cpu().numpy(), lo, 1e-8, "odd-grid adjoint")
    dfdx = sol.sensitivity(s, lam).cpu().numpy()
    _, do = model.sensitivity(so, lo, explicit=True)
    assert np.linalg.norm(dfdx - do) <= 1e-8 * np.linalg.norm(do)
