"""The design loop of Sec. 5 on the GPU (MMA, volume constraint, continuation, warm starts,
Q ramping) against the oracle's: the MMA update itself, a run of the whole loop, and the
heat-source ramp."""

import numpy as np
import pytest
import torch

import oracle
from oracle import design as odesign
from paper_1904_00182_amd import nc, inputs, workloads, design
from gpu_helpers import oracle_params, check_fields, to_dev, DEV

pytestmark = pytest.mark.gpu


def _start(m):
    """The paper's initial design: 0.05 in the design domain (Sec. 6.1), 1 in the solid
    block, 0 in the passive fluid."""
    return np.where(m.solid, 1.0, np.where(m.design, 0.05, 0.0))


def test_mma_update_matches_oracle():
    """Five successive MMA updates on the design elements of the 8x8x16 quarter cavity from
    random designs and derivatives (asymptotes initialised, then widened or narrowed),
    including a subproblem with lambda = 0 and one with no feasible point (lambda = inf):
    the same designs as the oracle's MMA to 1e-12 and the same multipliers to 1e-10."""
    p = workloads.benchmark_problem(8, 1e3)
    sol = nc.Solver(p, DEV)
    m = oracle.Model(oracle_params(p), np.zeros(sol.E))
    D = m.design
    r = inputs.rng(60)
    x = _start(m)
    x[D] = r.uniform(0.05, 0.95, D.sum())
    xg = to_dev(x)
    state = sol.mma_state()
    opt = oracle.MMA(int(D.sum()), move=0.2)
    for it, g in enumerate((0.01, 0.0, -5.0, 0.02, 50.0)):
        print("mma update", it, "g", g, flush=True)
        df = np.where(D, r.standard_normal(sol.E), 0.0)
        dg = np.where(D, np.abs(r.standard_normal(sol.E)) / D.sum(), 0.0)
        lam = sol.mma_update(it + 1, xg, to_dev(df), g, to_dev(dg), 0.2, state)
        xo, lo = opt.update(x[D], df[D], g, dg[D])
        x = x.copy()
        x[D] = xo
        xn = xg.cpu().numpy()
        assert np.abs(xn - x).max() <= 1e-12, (it, np.abs(xn - x).max())
        assert np.all(xn[~D] == _start(m)[~D])
        if np.isinf(lo):
            assert np.isinf(lam)
        elif lo == 0.0:
            assert lam == 0.0
        else:
            assert abs(lam - lo) <= 1e-10 * lo, (lam, lo)
    assert np.isinf(lo) and lam == np.inf


def test_design_loop_matches_oracle():
    """Six design iterations on the 8x8x16 quarter cavity (Gr 1e3, PDE filter, passive
    regions, volume fraction 0.05, move limit 0.2) with the continuation stage advanced every
    two iterations: per iteration the compliance and the volume fraction, and the designs,
    equal the oracle's loop within 1e-8."""
    p = workloads.benchmark_problem(8, 1e3)
    op = oracle_params(p)
    m = oracle.Model(op, np.zeros(p.nx * p.ny * p.nz))
    x0 = _start(m)
    xo, so, ho = odesign.optimize(op, x0, 6, every=2)
    xg, sg, hg = design.optimize(p, x0, 6, every=2, keep_designs=True)
    for it, (a, b) in enumerate(zip(hg, ho)):
        print(it, "gpu f", a["f"], "oracle f", b["f"], "frac", a["frac"], b["frac"], flush=True)
        assert abs(a["f"] - b["f"]) <= 1e-8 * abs(b["f"]), it
        assert abs(a["frac"] - b["frac"]) <= 1e-10, it
        assert np.abs(a["x"] - b["x"]).max() <= 1e-8, (it, np.abs(a["x"] - b["x"]).max())
        assert not a["ramped"]
    check_fields(sg.cpu().numpy(), so, 1e-8, "final state")


def test_q_ramp_reaches_the_direct_root():
    """The heat-source ramp of Sec. 5.4 (Q at 1/4, 1/2, 3/4, 1, each warm-started from the
    last) ends at the same root as the direct Newton solve."""
    p = workloads.benchmark_problem(8, 1e4, kappa_f=0.00206)
    sol = nc.Solver(p, DEV)
    m = oracle.Model(oracle_params(p), np.zeros(sol.E))
    x = to_dev(_start(m))
    sol.set_design(x)
    s1 = sol.solve_state()
    assert sol.last_info["status"] == nc.NC_OK
    s2 = torch.zeros_like(s1)
    info, ramped = design.solve_with_ramp(sol, p, x, s2, force_ramp=True)
    assert ramped and info["status"] == nc.NC_OK
    check_fields(s2.cpu().numpy(), s1.cpu().numpy(), 1e-10, "ramped vs direct")


def test_hybrid_ns_then_darcy_loop_matches_oracle():
    """The hybrid strategy of Sec. 6.4 (NS-D, the continuation of eq. contsch2) with its
    stages shortened to two iterations each: two Navier-Stokes / Brinkman stages (the
    solid's impermeability 1e5 interpolated with q_p), then the first Darcy stage, on the
    8x8x16 quarter cavity; per iteration the flow model, the compliance, the volume fraction
    and the designs equal the oracle's loop within 1e-8."""
    p = workloads.benchmark_problem(8, 1e3)
    op = oracle_params(p)
    m = oracle.Model(op, np.zeros(p.nx * p.ny * p.nz))
    x0 = _start(m)
    xo, so, ho = odesign.optimize(op, x0, 6, every=2, continuation=odesign.HYBRID_NS_D)
    xg, sg, hg = design.optimize(p, x0, 6, every=2, continuation=design.HYBRID_NS_D, keep_designs=True)
    for it, (a, b) in enumerate(zip(hg, ho)):
        print(it, a["model"], "gpu f", a["f"], "oracle f", b["f"], "frac", a["frac"], b["frac"],
              "krylov", a["state_krylov"], a["adjoint_krylov"], flush=True)
        assert a["model"] == b["model"]
        assert abs(a["f"] - b["f"]) <= 1e-8 * abs(b["f"]), it
        assert abs(a["frac"] - b["frac"]) <= 1e-10, it
        assert np.abs(a["x"] - b["x"]).max() <= 1e-8, (it, np.abs(a["x"] - b["x"]).max())
    assert [h["model"] for h in hg] == ["ns"] * 4 + ["darcy"] * 2
    check_fields(sg.cpu().numpy(), so, 1e-8, "final state")


def test_paper_optimisation_reaches_a_discrete_design():
    """The optimisation of Sec. 6.3 (eq. contsch1, here 5 x 20 iterations) on the 24x24x48
    quarter cavity at alpha 1e3 and 1e6, mixed precision: every state and adjoint solve
    converges (optimize raises otherwise), the volume constraint is active at the end, the
    design is nearly 0/1, the convection-dominated case ends with the lower compliance
    (Table tab:topoptperformance: 8.53 at alpha 1e3, 4.81 at 1e6), and each design is the
    better one at the alpha it was optimised for."""
    from paper_1904_00182_amd import design
    f, xs = {}, {}
    for alpha in (1e3, 1e6):
        xs[alpha], r = design.paper_optimisation(24, alpha, iterations=100, every=20, device=DEV)
        print(alpha, r, flush=True)
        assert abs(r["volume_fraction"] - 0.05) <= 2e-3, r
        assert r["gray_share"] <= 0.1, r
        f[alpha] = r["f_full_box"]
    assert f[1e6] < f[1e3]
    # the cross-check of Table tab:petscperformance: each design is best at its own alpha,
    # and a cold re-evaluation of a design agrees with its run's last compliance
    for a, b in ((1e3, 1e6), (1e6, 1e3)):
        own = design.paper_evaluate(24, a, xs[a], device=DEV)
        other = design.paper_evaluate(24, a, xs[b], device=DEV)
        print("analysis", a, own, other, flush=True)
        assert own < other
        assert abs(own - f[a]) <= 0.01 * f[a]
