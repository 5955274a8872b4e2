"""The multigrid preconditioner through nc_precondition: the single-workgroup bottom of
the V-cycle against the same cycle run with one launch per step, and the transposed
cycle against the forward one (with equal pre- and post-sweep counts on every level,
restriction = prolongation^T and coarse operators that are the exact transposes, the
transposed cycle is the adjoint of the forward cycle, so <u, M^-1 v> = <M^-T u, v>)."""

import numpy as np
import pytest
import torch

from paper_1904_00182_amd import nc, workloads
from gpu_helpers import DEV

pytestmark = pytest.mark.gpu

# relative agreement: float64 cycles differ only in summation order; float32 cycles by
# float32 rounding carried through a few dozen dependent steps
TOL = {nc.NC_FP64: 1e-11, nc.NC_MIXED: 3e-5}


def _solvers(grid, gr, precision):
    out = []
    for tail in (1, 0):
        p = workloads.problem(grid, gr, precision)
        p.coarse_tail = tail
        sol = nc.Solver(p, DEV)
        sol.set_design(workloads.design(grid, "blobs", 4, DEV))
        out.append(sol)
    s = out[0].solve_state()
    assert out[0].last_info["status"] == nc.NC_OK
    return out, s


def _vectors(n, seed):
    rng = np.random.default_rng(seed)
    return [torch.as_tensor(rng.standard_normal((n, 2)), device=DEV) for _ in range(2)]


def _rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("grid,gr", [((16, 8, 16), 1e3), ((32, 16, 32), 1e4)])
@pytest.mark.parametrize("precision", [nc.NC_FP64, nc.NC_MIXED], ids=["fp64", "mixed"])
def test_tail_cycle_matches_per_level_launches(grid, gr, precision):
    (tail, plain), s = _solvers(grid, gr, precision)
    v, _ = _vectors(tail.N, 11)
    for tr in (False, True):
        z1 = tail.precondition(s, v, transpose=tr)
        z0 = plain.precondition(s, v, transpose=tr)
        assert torch.isfinite(z1).all()
        assert _rel(z1, z0) < TOL[precision], (tr, _rel(z1, z0))
    # deterministic: a second application is bitwise identical
    assert torch.equal(tail.precondition(s, v), tail.precondition(s, v))


@pytest.mark.parametrize("grid,gr", [((16, 8, 16), 1e3), ((32, 16, 32), 1e4)])
@pytest.mark.parametrize("precision", [nc.NC_FP64, nc.NC_MIXED], ids=["fp64", "mixed"])
def test_transposed_cycle_is_the_adjoint(grid, gr, precision):
    sols, s = _solvers(grid, gr, precision)
    u, v = _vectors(sols[0].N, 12)
    for sol in sols:
        lhs = float((u * sol.precondition(s, v)).sum())
        rhs = float((sol.precondition(s, u, transpose=True) * v).sum())
        scale = float(u.norm() * sol.precondition(s, v).norm())
        assert abs(lhs - rhs) < TOL[precision] * scale, (lhs, rhs, scale)


def test_tail_cycle_leaves_solves_unchanged():
    """A linear solve at one state (the adjoint) takes the same FGMRES iterations either
    way, and the state and adjoint solutions agree to the mixed-precision accuracy.  (The
    iteration count of a cold Newton solve is not compared: its path through the loose
    first step is sensitive to rounding, e.g. one Newton step more or less.)"""
    (tail, plain), s = _solvers((32, 16, 32), 1e4, nc.NC_MIXED)
    g = tail.objective_grad()
    lams, infos = [], []
    for sol in (tail, plain):
        lams.append(sol.solve_adjoint(s, g))
        infos.append(dict(sol.last_info))
        assert infos[-1]["status"] == nc.NC_OK
    assert abs(infos[0]["krylov_its"] - infos[1]["krylov_its"]) <= 2, infos
    assert _rel(lams[0], lams[1]) < 1e-8
    states = []
    for sol in (tail, plain):
        states.append(sol.solve_state())
        assert sol.last_info["status"] == nc.NC_OK
    assert _rel(states[0], states[1]) < 1e-8
