"""Design loop of Sec. 5 on the GPU: volume-constrained minimisation of the thermal
compliance (eq. optprob) by MMA, with the step-wise continuation of Sec. 5.3 and the
solver practice of Sec. 5.4.

Per iteration (all arithmetic in the HIP library; this module only sequences the calls):
set the design (filter, passive regions, RAMP at the current continuation stage), solve the
state warm-started from the previous design's state, ramp the heat source Q if that Newton
solve fails, evaluate the compliance and its adjoint sensitivities, the volume constraint
and its gradient, and take one MMA step on the design elements (move limit of Sec. 6.1).
MMA sees f / f0, f0 being the first iteration's compliance (the paper states no scaling).
"""

import time

import torch

from . import nc

# eq. contsch1: (q_c, q_p, kappa_s) of the five stages, advanced every `every` iterations
CONTINUATION = ((0.881, 8.0, 1e-5), (8.81, 8.0, 1e-5), (88.1, 8.0, 1e-5), (88.1, 98.0, 1e-6), (881.0, 998.0, 1e-7))
Q_RAMP = (0.25, 0.5, 0.75, 1.0)


def stage_problem(problem, it, every, continuation=CONTINUATION):
    q_c, q_p, kappa_s = continuation[min(it // every, len(continuation) - 1)]
    return nc.copy_problem(problem, q_c=q_c, q_p=q_p, kappa_s=kappa_s)


def solve_with_ramp(sol, problem, x, s, force_ramp=False):
    """State solve for design x warm-started from s (updated in place).  If Newton fails
    (or force_ramp), the heat source is ramped through Q_RAMP from the same warm start,
    each stage starting from the last.  Returns (info of the final solve, ramped?)."""
    s0 = s.clone()
    if not force_ramp:
        sol.solve_state(out=s)
        if sol.last_info["status"] == nc.NC_OK:
            return dict(sol.last_info), False
    s.copy_(s0)
    for frac in Q_RAMP:
        sol.set_problem(nc.copy_problem(problem, Q=frac * problem.Q))
        sol.set_design(x)
        sol.solve_state(out=s)
    sol.set_problem(problem)
    sol.set_design(x)
    return dict(sol.last_info), True


def optimize(problem, x0, iterations, g_star=0.05, move=0.2, every=100, continuation=CONTINUATION, device="cuda:0",
             sol=None, log=None, keep_designs=False):
    """Runs the design loop from the raw design x0 ([E]; passive entries are kept).
    Returns (x, s, history) with per iteration: compliance f, volume fraction, MMA
    multiplier, Newton and FGMRES counts, whether Q was ramped, and seconds."""
    sol = sol or nc.Solver(stage_problem(problem, 0, every, continuation), device)
    x = torch.as_tensor(x0, dtype=torch.float64, device=sol.device).clone().contiguous()
    s = torch.zeros((sol.N, 5), dtype=torch.float64, device=sol.device)
    state = sol.mma_state()
    f0 = None
    stage = None
    hist = []
    for it in range(iterations):
        t0 = time.perf_counter()
        p = stage_problem(problem, it, every, continuation)
        st = min(it // every, len(continuation) - 1)
        if st != stage:
            sol.set_problem(p)
            stage = st
        sol.set_design(x)
        info, ramped = solve_with_ramp(sol, p, x, s)
        if info["status"] != nc.NC_OK:
            raise RuntimeError(f"state solve failed at design iteration {it}: {info}")
        f = sol.objective(s)
        lam = sol.solve_adjoint(s, sol.objective_grad(s))
        ainfo = dict(sol.last_info)
        if ainfo["status"] != nc.NC_OK:
            raise RuntimeError(f"adjoint solve failed at design iteration {it}: {ainfo}")
        dfdx = sol.objective_sensitivity(s, lam)
        frac, dv = sol.volume()
        if f0 is None:
            f0 = f
        mult = sol.mma_update(it + 1, x, dfdx / f0, frac - g_star, dv, move, state)
        torch.cuda.synchronize(sol.device)
        h = dict(it=it, f=f, frac=frac, lam=mult, ramped=ramped, newton=info["newton_its"],
                 state_krylov=info["krylov_its"], adjoint_krylov=ainfo["krylov_its"], state_s=info["t_total"],
                 adjoint_s=ainfo["t_total"], seconds=time.perf_counter() - t0)
        if keep_designs:
            h["x"] = x.cpu().numpy().copy()
        hist.append(h)
        if log:
            log(h)
    return x, s, hist
