"""Design loop of Sec. 5 on the GPU: volume-constrained minimisation of the thermal
compliance (eq. optprob) by MMA, with the step-wise continuation of Sec. 5.3 and the
solver practice of Sec. 5.4.

Per iteration (all arithmetic in the HIP library; this module only sequences the calls):
set the design (filter, passive regions, RAMP at the current continuation stage), solve the
state warm-started from the previous design's state, ramp the heat source Q if that Newton
solve fails, evaluate the compliance and its adjoint sensitivities, the volume constraint
and its gradient, and take one MMA step on the design elements (move limit of Sec. 6.1).
MMA sees f / f0, f0 being the first iteration's compliance (the paper states no scaling).
The continuation can switch the flow model between stages: the hybrid strategy of Sec. 6.4
(eq. contsch2) runs its first stages with the Navier-Stokes / Brinkman model.
"""

import time

import torch

from . import nc

# eq. contsch1: (q_c, q_p, kappa_s) of the five stages, advanced every `every` iterations
CONTINUATION = ((0.881, 8.0, 1e-5), (8.81, 8.0, 1e-5), (88.1, 8.0, 1e-5), (88.1, 98.0, 1e-6), (881.0, 998.0, 1e-7))
# eq. contsch2, the hybrid strategy of Sec. 6.4 (NS-D of Table tab:hybridapproaches): two
# stages with the Navier-Stokes / Brinkman model (q_p and kappa_s interpolate the solid's
# impermeability there), then three with the Darcy model
HYBRID_NS_D = (("ns", 0.881, 8.0, 1e5), ("ns", 8.81, 8.0, 1e5), ("darcy", 88.1, 8.0, 1e-5),
               ("darcy", 88.1, 98.0, 1e-6), ("darcy", 881.0, 998.0, 1e-7))
Q_RAMP = (0.25, 0.5, 0.75, 1.0)
# solver settings of the Navier-Stokes stages: damped node-block Jacobi (the undamped
# smoother diverges on the saddle-point blocks) and the adjoint target that gives the
# multipliers to about 1e-10
NS_SETTINGS = dict(smooth_omega=0.7, adjoint_rtol=1e-12)


def stage(continuation, it, every):
    """(model kind, q_c, q_p, kappa_s) of iteration it; plain triples are Darcy stages."""
    st = continuation[min(it // every, len(continuation) - 1)]
    return tuple(st) if len(st) == 4 else ("darcy",) + tuple(st)


def stage_problem(problem, it, every, continuation=CONTINUATION):
    kind, q_c, q_p, kappa_s = stage(continuation, it, every)
    extra = NS_SETTINGS if kind == "ns" else {}
    return nc.copy_problem(problem, q_c=q_c, q_p=q_p, kappa_s=kappa_s, **extra)


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
    Returns (x, s, history) with per iteration: flow model, compliance f, volume fraction,
    MMA multiplier, Newton and FGMRES counts, whether Q was ramped, and seconds.

    A continuation may name the flow model per stage (the hybrid strategy of Sec. 6.4):
    Navier-Stokes stages solve with an nc_ns context; the Darcy context `sol` always serves
    the volume constraint and MMA (they depend on the filtered design only).  A change of
    model starts the state from zero."""
    stages = [stage(continuation, k * every, every) for k in range(len(continuation))]
    first_darcy = next((k for k, st in enumerate(stages) if st[0] == "darcy"), 0)
    sol = sol or nc.Solver(stage_problem(problem, first_darcy * every, every, continuation), device)
    nsol = None
    x = torch.as_tensor(x0, dtype=torch.float64, device=sol.device).clone().contiguous()
    s = torch.zeros((sol.N, 5), dtype=torch.float64, device=sol.device)
    state = sol.mma_state()
    f0 = None
    current = None
    hist = []
    for it in range(iterations):
        t0 = time.perf_counter()
        p = stage_problem(problem, it, every, continuation)
        kind = stage(continuation, it, every)[0]
        st = min(it // every, len(continuation) - 1)
        if kind == "ns" and nsol is None:
            nsol = nc.NSSolver(p, sol.device)
        solver = nsol if kind == "ns" else sol
        if current is None or st != current[1]:
            if current is None or kind != current[0]:
                s.zero_()
            solver.set_problem(p)
            current = (kind, st)
        solver.set_design(x)
        info, ramped = solve_with_ramp(solver, p, x, s)
        if info["status"] != nc.NC_OK:
            raise RuntimeError(f"state solve failed at design iteration {it}: {info}")
        f = solver.objective(s)
        lam = solver.solve_adjoint(s, solver.objective_grad(s))
        ainfo = dict(solver.last_info)
        if ainfo["status"] != nc.NC_OK:
            raise RuntimeError(f"adjoint solve failed at design iteration {it}: {ainfo}")
        if kind == "ns":
            dfdx = solver.sensitivity(s, lam)
            sol.set_design(x)
        else:
            dfdx = solver.objective_sensitivity(s, lam)
        frac, dv = sol.volume()
        if f0 is None:
            f0 = f
        mult = sol.mma_update(it + 1, x, dfdx / f0, frac - g_star, dv, move, state)
        torch.cuda.synchronize(sol.device)
        h = dict(it=it, model=kind, f=f, frac=frac, lam=mult, ramped=ramped, newton=info["newton_its"],
                 state_krylov=info["krylov_its"], adjoint_krylov=ainfo["krylov_its"], state_s=info["t_total"],
                 adjoint_s=ainfo["t_total"], krylov_f64=max(info.get("krylov_f64", 0), ainfo.get("krylov_f64", 0)),
                 seconds=time.perf_counter() - t0)
        if keep_designs:
            h["x"] = x.cpu().numpy().copy()
        hist.append(h)
        if log:
            log(h)
    return x, s, hist


def paper_optimisation(n, alpha, iterations=500, every=100, precision=nc.NC_MIXED, device="cuda:0", log=None):
    """The optimisation of Sec. 6.3 on the benchmark of Sec. 6.1 with n x n x 2n elements of
    the quarter cavity: the paper's initial design, eq. contsch1 advanced every `every`
    iterations, g* = 0.05, move limit 0.2, the Table tab:2 permeability for alpha.  Returns
    (final raw design, summary) with the thermal compliance of the quarter model and of the
    full symmetric box (four quarters), the volume fraction, the share of design elements
    with intermediate density (0.1 < gamma < 0.9), the iteration from which Krylov ran in
    float64 (mixed precision), and the seconds taken."""
    from . import workloads
    p = workloads.benchmark_problem(n, alpha, precision)
    x0 = workloads.benchmark_start_design(p, device)
    torch.cuda.synchronize(device)
    t0 = time.perf_counter()
    x, _, hist = optimize(p, x0, iterations, every=every, continuation=CONTINUATION, device=device, log=log)
    torch.cuda.synchronize(device)
    wall = time.perf_counter() - t0
    sol = nc.Solver(stage_problem(p, iterations - 1, every), device)
    sol.set_design(x)
    gam = sol.gamma()
    _, dv = sol.volume()
    design = dv != 0
    gray = float(((gam > 0.1) & (gam < 0.9) & design).sum()) / max(1, int(design.sum()))
    sol.close()
    f = hist[-1]["f"]
    return x, {"grid": [p.nx, p.ny, p.nz], "alpha": alpha, "iterations": iterations,
               "precision": "f32+f64" if precision == nc.NC_MIXED else "f64",
               "f_quarter": f, "f_full_box": 4.0 * f, "volume_fraction": hist[-1]["frac"], "gray_share": gray,
               "float64_krylov_from_iteration": next((h["it"] for h in hist if h["krylov_f64"]), None),
               "ramped_iterations": sum(1 for h in hist if h["ramped"]), "wall_s": wall}


def paper_evaluate(n, alpha, x, precision=nc.NC_MIXED, device="cuda:0"):
    """Compliance of the full box (four quarters) of the raw design x on the n x n x 2n
    benchmark at alpha, with the penalties of the continuation's last stage: the cross-check
    of optimised designs under every operating condition (Table tab:petscperformance).  The
    state solve starts cold, with the Q ramp if Newton fails."""
    from . import workloads
    p = stage_problem(workloads.benchmark_problem(n, alpha, precision), len(CONTINUATION) - 1, 1)
    sol = nc.Solver(p, device)
    sol.set_design(x)
    s = torch.zeros((sol.N, 5), dtype=torch.float64, device=device)
    info, _ = solve_with_ramp(sol, p, x, s)
    if info["status"] != nc.NC_OK:
        raise RuntimeError(f"state solve failed evaluating a design at alpha {alpha:g}: {info}")
    f = sol.objective(s)
    sol.close()
    return 4.0 * f
