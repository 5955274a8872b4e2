#!/usr/bin/env python3
"""Benchmark of the natural-convection state + adjoint solve on one MI355X.

One step = the whole hot path for one design on the 128 x 64 x 128 cavity (1,048,576
elements, 5,408,325 dofs), Gr = 1e4, filtered-noise 0/1 design, mixed precision:
cold-start Newton state solve (float64 residual and update, float32 FGMRES + multigrid
inner solves), the objective gradient, the adjoint solve (float32 inner, float64
refinement) and the sensitivities through RAMP and the filter.  Inputs are resident in
HBM before the timed region.

Printed: one JSON line with the step time (the metric is "state+adjoint solve s at 1M
elems", lower is better), the roofline of the dominant kernel from live HIP-event timing
on the solver's stream (vector-ALU bound for the operator kernels, HBM bound for the
streaming ones), operator GDoF/s, and the float64 CPU oracle timed on a small sample of
the same workload on this host.  --report FILE adds the extended measurements.
"""

import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = {4: 157.3, 8: 78.6}     # MI355X vector peaks, float32 and float64

# Flops of one operator launch per finest-grid element and node: the element
# linearisation (279) plus the element apply, and the node-level assembly and finishing.
# The element figures are counted on the element code by tests/native/flop_count.cpp
# (checked by tests/test_flop_count.py).
FLOPS_PER_ELEM = {"jv": 279 + 524, "jtw": 279 + 593, "smooth": 279 + 524, "smooth_T": 279 + 593,
                  "pt_residual": 279 + 524}
FLOPS_PER_NODE = {"jv": 16, "jtw": 16, "smooth": 26, "smooth_T": 26, "pt_residual": 16}

# timed classes that are one kernel at one grid size, their kernel symbols (tile template
# arguments elided) and the pattern of their names in rocprofv3 output
SINGLE_KERNEL_CLASSES = ("smooth", "smooth_T", "pt_residual", "jv", "jtw", "mdot", "maxpy")
KERNEL_NAMES = {
    "jv": "zmarch_kernel<JvOp<{t},2,0>,..,1> (Krylov operator: (P, T) block of J)",
    "jtw": "zmarch_kernel<JtwOp<{t},2,0>,..,1> (Krylov operator: (P, T) block of J^T)",
    "smooth": "zmarch_kernel<JvOp<{t},2,2>,..,1> (finest-grid block-Jacobi sweep)",
    "smooth_T": "zmarch_kernel<JtwOp<{t},2,2>,..,1> (finest-grid transposed block-Jacobi sweep)",
    "pt_residual": "zmarch_kernel<JvOp/JtwOp<{t},2,1>,..,1> (finest-grid multigrid residual)",
    "mdot": "mdot_kernel<{t}> (FGMRES multi-dot)",
    "maxpy": "maxpy_kernel<{t}> (FGMRES multi-axpy)",
}
PROFILE_NAMES = {
    "jv": r"zmarch_kernel<JvOp<{t}, 2, 0, false>, \d+, 1>", "jtw": r"zmarch_kernel<JtwOp<{t}, 2, 0, false>, \d+, 1>",
    "smooth": r"zmarch_kernel<JvOp<{t}, 2, 2, false>, \d+, 1>", "smooth_T": r"zmarch_kernel<JtwOp<{t}, 2, 2, false>, \d+, 1>",
    "pt_residual": r"zmarch_kernel<JvOp<{t}, 2, 1, false>, \d+, 1>", "mdot": r"mdot_kernel<{t}>", "maxpy": r"maxpy_kernel<{t}>",
}
# kernel sources whose hash must match the one recorded with the counter runs: every
# source of the library

def measured_counters(cls, tname):
    """(HBM bytes, VALU instructions) per launch of the class's kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE calibrated; SQ_INSTS_VALU), or (None, None)
    when there is none or the kernel sources have changed since the counters were taken."""
    rec = _counter_record()
    if rec is None:
        return None, None
    import re
    pat = re.compile(PROFILE_NAMES[cls].format(t=tname) + "$")
    for name, v in rec["kernels"].items():
        if pat.match(name):
            return round(v["fetch_bytes"] + v["write_bytes"]), v.get("valu_insts")
    return None, None


def _counter_record():
    """The committed counter summary, if the sources it was taken with are unchanged: the
    record lists every kernel source file of the library at the time (all of them go into
    the operator kernels' build) and their SHA-256; a file added later, which those kernels
    do not include, does not invalidate it."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_cavity128x64x128_mixed.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    files = rec.get("source_files")
    if not files or not all(os.path.exists(os.path.join(ROOT, f)) for f in files):
        return None
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if rec.get("source_sha256") != h.hexdigest():
        return None
    return rec


def measured_traffic(cls, tname):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) of the class's kernel from
    the committed counter summary, or None when there is none or the kernel sources have
    changed since the counters were taken."""
    return measured_counters(cls, tname)[0]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cavity128mixed")
    ap.add_argument("--apply-iters", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-grid", default="24,12,24")
    ap.add_argument("--no-fp64-leg", action="store_true", help="skip the float64 solve of the same workload")
    ap.add_argument("--no-oracle-pair", action="store_true",
                    help="skip the oracle-vs-GPU float64 pair on the 32x16x32 cavity")
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-design-loop", action="store_true", help="skip the design-loop timing on the 80x80x160 benchmark")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving run")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--serving-load", type=float, default=1.5,
                    help="arrival rate as a multiple of the measured one-at-a-time capacity")
    ap.add_argument("--design-iters", type=int, default=10)
    ap.add_argument("--no-ns", action="store_true", help="skip the Navier-Stokes / Brinkman model's timings")
    ap.add_argument("--hybrid-iters", type=int, default=4, help="design iterations per stage of the hybrid NS-D run")
    ap.add_argument("--paper-runs", type=int, default=0,
                    help="also run the paper's 500-iteration optimisation of Sec. 6.3 on the n x n x 2n quarter cavity "
                         "for each --paper-alphas value (n = 160 is the paper's mesh; 0 skips it)")
    ap.add_argument("--paper-alphas", default="1e3,1e4,1e5,1e6")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--report", default=None,
                    help="also write extended measurements (operator sweep, float64 baseline, warm re-solve, "
                         "oracle phases, serving) as JSON to this file")
    ap.add_argument("--report-requests", type=int, default=128)
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="also run one device copy of this many MiB (a kernel of known traffic for counter scaling)")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def time_apply(sol, torch, dtype, transpose, iters, pairs):
    """Average duration of the five-field Jacobian apply with HIP events on the solver's
    stream, rotating over `pairs` input/output buffers (working set beyond the L2 and
    Infinity Cache)."""
    N = sol.N
    gen = torch.Generator(device=sol.device).manual_seed(1)
    vs = [torch.randn((N, 5), dtype=dtype, device=sol.device, generator=gen) for _ in range(pairs)]
    ys = [torch.empty_like(vs[0]) for _ in range(pairs)]
    from paper_1904_00182_amd import nc
    lib = sol.lib
    if dtype == torch.float64:
        f = lib.nc_jacT_apply if transpose else lib.nc_jac_apply
    else:
        f = lib.nc_jacT_apply_f32 if transpose else lib.nc_jac_apply_f32
    import ctypes
    ptrs = [(ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(y.data_ptr())) for v, y in zip(vs, ys)]
    for k in range(pairs):
        f(sol.ctx, *ptrs[k])
    torch.cuda.synchronize()
    st = sol.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for k in range(iters):
        f(sol.ctx, *ptrs[k % pairs])
    e1.record(st)
    e1.synchronize()
    return e0.elapsed_time(e1) / iters * 1e-3


def cpu_baseline(args, E_target):
    """The float64 oracle (assembled complex-step Jacobian, SuperLU) on a bounded sample of
    the same workload family, scaled linearly in the element count (a lower bound for a
    direct solver, whose cost grows faster than linearly)."""
    import numpy as np
    import oracle
    from paper_1904_00182_amd import inputs
    nx, ny, nz = (int(v) for v in args.cpu_grid.split(","))
    p = oracle.Params(nx, ny, nz, alpha=1e4, kappa_f=0.00206)
    F = oracle.cone_filter_matrix(oracle.Mesh(p), 2.0)
    x = (F @ inputs.uniform_design(nx * ny * nz, 2) >= 0.5).astype(np.float64)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    m = oracle.Model(p, x)
    s, _ = m.solve_state()
    lam = m.solve_adjoint(s, m.dfds())
    m.sensitivity(s, lam)
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    E = nx * ny * nz
    return {
        "value": round(wall * E_target / E, 3),
        "unit": "s",
        "cores": max(1, int(round(cpu / wall))),
        "kind": "oracle",
        "sample": f"state+adjoint+sensitivity on the {nx}x{ny}x{nz} cavity ({E} elements, Gr 1e4, "
                  f"thresholded filtered-noise design): {wall:.2f} s wall, scaled x{E_target / E:.1f} "
                  f"linearly to {E_target} elements",
        "cpu_model": _cpu_model(),
        "host_cores_available": len(os.sched_getaffinity(0)),
        "phases_s": {k: round(v, 3) for k, v in m.timing.items()},
    }


def nc_status(code):
    from paper_1904_00182_amd import nc
    return nc.load().nc_status_string(code).decode()


def field_errors(a, b, names):
    """Per field: relative l2 error and element-wise max|a - b| / max|b|."""
    import torch
    out = {}
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    for k, nm in enumerate(names):
        if nm is None:
            continue
        d = (a[:, k] - b[:, k]).abs()
        nb = float(torch.linalg.vector_norm(b[:, k]))
        mb = float(b[:, k].abs().max())
        out[nm] = {"rel_l2": float(torch.linalg.vector_norm(d)) / nb if nb > 0 else None,
                   "rel_max": float(d.max()) / mb if mb > 0 else None}
    return out


def fp64_leg(args, mixed_result):
    """The plain float64 GPU solve of the same workload (float64 operator, multigrid and
    FGMRES): step time and iteration counts, and the per-field error of the mixed-precision
    results against it."""
    import torch
    from paper_1904_00182_amd import nc, workloads
    dev = "cuda:0"
    p, x, cfg = workloads.config("cavity128", dev)
    sol = nc.Solver(p, dev)
    sol.set_design(x)
    g = sol.objective_grad()
    N = sol.N
    s = torch.zeros((N, 5), dtype=torch.float64, device=dev)
    lam = torch.zeros_like(s)
    info = []

    def step():
        sol.set_design(x)
        s.zero_()
        sol.solve_state(out=s)
        i1 = dict(sol.last_info)
        sol.solve_adjoint(s, g, out=lam)
        i2 = dict(sol.last_info)
        if i1["status"] != nc.NC_OK or i2["status"] != nc.NC_OK:
            raise RuntimeError(f"float64 solve did not converge: {i1['status']} {i2['status']}")
        info.append((i1, i2))
        return sol.sensitivity(s, lam)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.fp64_steps):
        dfdx = step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.fp64_steps
    i1, i2 = info[-1]
    sm, lm, gm = mixed_result
    out = {
        "workload": "the same 128x64x128 cavity and design, float64 throughout",
        "ms_per_step": round(t * 1e3, 3), "steps": args.fp64_steps,
        "state_status": nc_status(i1["status"]), "adjoint_status": nc_status(i2["status"]),
        "newton_its": i1["newton_its"], "state_krylov_its": i1["krylov_its"],
        "adjoint_krylov_its": i2["krylov_its"], "adjoint_refinements": i2["refine_its"],
        "mixed_speedup": None,
        "mixed_vs_fp64": {
            "state": field_errors(sm, s, ("u", "v", "w", "P", "T")),
            "adjoint": field_errors(lm, lam, (None, None, None, "P", "T")),
            "dfdx": field_errors(gm.reshape(-1, 1), dfdx.reshape(-1, 1), ("dfdx",)),
        },
    }
    sol.close()
    del sol
    torch.cuda.empty_cache()
    log(args, "fp64 leg", out)
    return out


def design_loop_timing(args):
    """Design iterations of Sec. 5 on the paper's performance-study mesh (Sec. 6.2): the
    80x80x160 quarter cavity (1,024,000 elements, 1,056,321 nodes), heat-source block,
    passive regions, PDE filter R = 2.5, constant penalties q_c = 8.81, q_p = 8 (as in that
    study), kappa_s = 1e-5, from the paper's initial design 0.05.  Each iteration: design
    chain, warm-started Newton state solve, adjoint, sensitivities, volume constraint, MMA.
    Gr 1e3 in mixed precision, Gr 1e6 in float64 and in mixed precision (with the float64
    Krylov reserve of that regime)."""
    import torch
    from paper_1904_00182_amd import design, nc, workloads
    dev = "cuda:0"
    out = {"workload": "quarter cavity 80x80x160 of the paper's benchmark (Sec. 6.1), Q = 1e4 block, PDE filter R = 2.5, "
                       "q_c = 8.81, q_p = 8, kappa_s = 1e-5, g* = 0.05, move 0.2, start 0.05",
           "iterations": args.design_iters}
    for alpha, prec in ((1e3, nc.NC_MIXED), (1e6, nc.NC_FP64), (1e6, nc.NC_MIXED)):
        p = workloads.benchmark_problem(80, alpha, prec, kappa_s=1e-5, q_c=8.81, q_p=8.0)
        x0 = workloads.benchmark_start_design(p, dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, hist = design.optimize(p, x0, args.design_iters, every=10 ** 9, continuation=((8.81, 8.0, 1e-5),),
                                     device=dev)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        warm = hist[1:]
        key = f"gr{alpha:g}" + ("_mixed" if alpha >= 1e5 and prec == nc.NC_MIXED else "")
        out[key] = {
            "precision": "f32+f64" if prec == nc.NC_MIXED else "f64",
            "s_per_iteration": round(sum(h["seconds"] for h in warm) / len(warm), 4),
            "state_s_per_iteration_warm": round(sum(h["state_s"] for h in warm) / len(warm), 4),
            "state_s_first_cold": round(hist[0]["state_s"], 4),
            "adjoint_s_per_iteration": round(sum(h["adjoint_s"] for h in warm) / len(warm), 4),
            "newton_per_iteration_warm": round(sum(h["newton"] for h in warm) / len(warm), 2),
            "fgmres_per_newton_step_warm": round(sum(h["state_krylov"] for h in warm) / max(1, sum(h["newton"] for h in warm)), 2),
            "ramped": sum(1 for h in hist if h["ramped"]),
            "float64_krylov_from_iteration": next((h["it"] for h in hist if h["krylov_f64"]), None),
            "f_first_last": [hist[0]["f"], hist[-1]["f"]],
            "volume_last": hist[-1]["frac"],
            "wall_s": round(wall, 3),
        }
        log(args, "design loop", key, out[key])
    out["paper_context"] = ("state-solver time per optimisation iteration at 80x80x160, warm-started, 250 iterations: "
                            "Gr 1e3 37.29 s on 16 and 1.25 s on 640 Xeon E5-2680v2 cores; Gr 1e6 44.77 s and 1.65 s "
                            "(Table tab:jessperformance1); other hardware and 1e-4 / 1e-5 tolerances, context only")
    return out


# Table tab:topoptperformance: final objective and hours on 500 CPUs after 500 iterations
# on the 160 x 160 x 320 quarter cavity
PAPER_OPTIMISATION = {1e3: (8.53, 5.5), 1e4: (8.28, 2.8), 1e5: (6.67, 3.5), 1e6: (4.81, 4.2)}


def paper_runs(args):
    """The paper's optimisation of Sec. 6.3 (eq. contsch1, 500 iterations, mixed precision)
    on the n x n x 2n quarter cavity, per alpha: the final compliance of the full box (four
    quarters) against Table tab:topoptperformance, and the wall time on this GPU."""
    from paper_1904_00182_amd import design
    out = {"workload": f"quarter cavity {args.paper_runs}x{args.paper_runs}x{2 * args.paper_runs} of Sec. 6.1, eq. "
                       "contsch1 every 100 iterations, g* = 0.05, move 0.2, start 0.05, PDE filter R = 2.5",
           "paper": "Table tab:topoptperformance: 160x160x320, 500 iterations, 500 CPUs", "runs": []}
    alphas = [float(v) for v in args.paper_alphas.split(",")]
    designs = {}
    for a in alphas:
        def lg(h, a=a):
            if h["it"] % 100 == 99:
                log(args, "paper run", f"alpha {a:g} it {h['it']} f {h['f']:.4f}")
        designs[a], r = design.paper_optimisation(args.paper_runs, a, log=lg)
        ref = PAPER_OPTIMISATION.get(a)
        if ref is not None:
            r["paper_f"] = ref[0]
            r["paper_hours_500_cpus"] = ref[1]
            r["f_full_box_vs_paper"] = round(r["f_full_box"] / ref[0] - 1.0, 4)
        out["runs"].append(r)
        log(args, "paper run", r)
    if len(alphas) > 1:
        # every design under every operating condition (Table tab:petscperformance): rows are
        # the analysis alpha, columns the alpha the design was optimised for
        out["cross_check_alphas"] = alphas
        out["cross_check_f_full_box"] = []
        for a in alphas:
            row = [design.paper_evaluate(args.paper_runs, a, designs[b]) for b in alphas]
            out["cross_check_f_full_box"].append(row)
            log(args, "paper cross-check", f"alpha {a:g}", [round(v, 3) for v in row])
    return out


def ns_timing(args):
    """The Navier-Stokes / Brinkman flow model (the full-flow model of the hybrid strategy,
    Sec. 6.4) on the bench workload's grid and design: cold and warm state solves, the
    adjoint, the float64 operator apply (its assembled node-block Jacobian is HBM-bound),
    and design iterations of the hybrid NS-D continuation (eq. contsch2) on the paper's
    80x80x160 quarter cavity, Navier-Stokes stage against Darcy stage."""
    import torch
    from paper_1904_00182_amd import design, nc, workloads
    dev = "cuda:0"
    p, x, _ = workloads.config(args.workload)
    pn = nc.copy_problem(p, kappa_s=1e5, q_p=8.0, **design.NS_SETTINGS)
    sol = nc.NSSolver(pn, dev)
    sol.set_design(x)
    out = {"workload": f"{args.workload} grid and design with the Navier-Stokes / Brinkman model (solid impermeability "
                       f"1e5, q_p 8), Gr {p.alpha:g}, float64 Krylov with a "
                       + ("float32" if p.precision == nc.NC_MIXED else "float64") + " multigrid preconditioner"}
    s = sol.solve_state()
    torch.cuda.synchronize()
    for rep in range(2):
        t0 = time.perf_counter()
        s = sol.solve_state()
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        i_s = dict(sol.last_info)
        g = sol.objective_grad(s)
        t0 = time.perf_counter()
        lam = sol.solve_adjoint(s, g)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        i_a = dict(sol.last_info)
    out.update({"state_status": nc_status(i_s["status"]), "adjoint_status": nc_status(i_a["status"]),
                "state_s": round(ts, 4), "adjoint_s": round(ta, 4), "newton_its": i_s["newton_its"],
                "state_krylov_per_newton_step": i_s["hist_krylov"], "adjoint_krylov_its": i_a["krylov_its"],
                "adjoint_rel_res": i_a["rel_res"], "assembly_and_setup_s": round(i_s["t_setup"], 4),
                "levels": i_s["levels"], "objective": sol.objective(s)})
    # float64 operator apply y = J~ v on the assembled Jacobian (27 x 25 entries per node)
    N = sol.N
    v = torch.randn((N, 5), dtype=torch.float64, device=dev)
    y = torch.empty_like(v)
    lib = nc.load()
    ptr = lambda t: nc.ctypes.c_void_p(t.data_ptr())
    for _ in range(3):
        lib.nc_ns_jac_apply(sol.ctx, ptr(v), ptr(y))
    iters = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        lib.nc_ns_jac_apply(sol.ctx, ptr(v), ptr(y))
    e1.record()
    torch.cuda.synchronize()
    t_apply = e0.elapsed_time(e1) / iters * 1e-3
    nbytes = (27 * 25 * 8 + 2 * 5 * 8) * N
    out["operator_f64"] = {"us": round(t_apply * 1e6, 1), "gdof_s": round(5 * N / t_apply / 1e9, 2),
                           "algorithmic_bytes": nbytes, "gb_s": round(nbytes / t_apply / 1e9, 1),
                           "hbm_frac": round(nbytes / t_apply / 8e12, 3),
                           "bytes_per_node": "27 x 25 float64 matrix entries + 5 read + 5 written"}
    log(args, "navier-stokes", out)
    sol.close()
    del sol
    torch.cuda.empty_cache()
    # hybrid NS-D design iterations on the 80x80x160 quarter cavity
    pb = workloads.benchmark_problem(80, 1e3, nc.NC_MIXED, kappa_s=1e-5, q_c=8.81, q_p=8.0)
    x0 = workloads.benchmark_start_design(pb, dev)
    every = max(2, args.hybrid_iters)
    cont = (("ns", 8.81, 8.0, 1e5), ("darcy", 88.1, 8.0, 1e-5))
    torch.cuda.synchronize()
    _, _, hist = design.optimize(pb, x0, 2 * every, every=every, continuation=cont, device=dev)
    hy = {"workload": "quarter cavity 80x80x160 (Sec. 6.1), Gr 1e3, PDE filter R = 2.5, Q = 1e4 block; stages of "
                      f"{every} iterations: Navier-Stokes (q_c 8.81, q_p 8, impermeability 1e5), then Darcy "
                      "(q_c 88.1, q_p 8, kappa_s 1e-5); each stage's first iteration starts cold and is excluded"}
    for kind in ("ns", "darcy"):
        hs = [h for h in hist if h["model"] == kind][1:]
        hy[kind] = {"s_per_iteration": round(sum(h["seconds"] for h in hs) / len(hs), 4),
                    "state_s": round(sum(h["state_s"] for h in hs) / len(hs), 4),
                    "adjoint_s": round(sum(h["adjoint_s"] for h in hs) / len(hs), 4),
                    "newton_per_iteration": round(sum(h["newton"] for h in hs) / len(hs), 2),
                    "fgmres_per_newton_step": round(sum(h["state_krylov"] for h in hs) / max(1, sum(h["newton"] for h in hs)), 2)}
    hy["ns_over_darcy"] = round(hy["ns"]["s_per_iteration"] / hy["darcy"]["s_per_iteration"], 2)
    hy["paper_context"] = ("hybrid NS-D at alpha 1e3 (Table tab:topoptperformancehybrid, other hardware): Navier-Stokes "
                           "200 iterations 20.0 h, Darcy 300 iterations 1.5 h, i.e. 360 s and 18 s per iteration")
    out["hybrid_design"] = hy
    log(args, "hybrid design", hy)
    return out


def pde_filter_timing(args):
    """The PDE (Helmholtz) density filter of Sec. 5.1 (radius 2.5 element lengths) on the
    128x64x128 grid: time of one application (nc_filter_apply: element-to-node load, the
    planned Chebyshev steps, node-to-element average) with HIP events on the solver's
    stream, and its HBM fraction by algorithmic bytes (per step: read the direction, the
    iterate and the residual, write the iterate, the residual and the next direction)."""
    import torch
    from paper_1904_00182_amd import nc, workloads
    dev = "cuda:0"
    p, x, cfg = workloads.config("cavity128pde", dev)
    sol = nc.Solver(p, dev)
    y = torch.empty_like(x)
    for _ in range(3):
        sol.filter_apply(x)
    torch.cuda.synchronize()
    st = sol.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    import ctypes
    xp, yp = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    reps = 20
    e0.record(st)
    for _ in range(reps):
        sol.lib.nc_filter_apply(sol.ctx, 0, xp, yp)
    e1.record(st)
    e1.synchronize()
    t = e0.elapsed_time(e1) / reps * 1e-3
    N, E = sol.N, sol.E
    # radius 2.5: 29 Chebyshev steps (bounds from the closed-form symbol; see the library)
    steps = 29
    algo = 8.0 * (steps * 6 * N + (E + 3 * N) + (2 * N + E))
    sol.close()
    out = {"grid": [p.nx, p.ny, p.nz], "radius": 2.5, "apply_us": round(t * 1e6, 2), "chebyshev_steps": steps,
           "algorithmic_bytes": algo, "hbm_frac": round(algo / t / 1e9 / HBM_PEAK_GBS, 4)}
    log(args, "pde filter", out)
    return out


def oracle_pair(args):
    """Like for like on the 32x16x32 cavity (Gr 1e3, thresholded filtered-noise design,
    seed 1): the float64 oracle (assembled complex-step Jacobian, SuperLU) and the float64
    GPU solve of the same problem, timed in the same run, with the GPU's per-field error
    against the oracle."""
    import numpy as np
    import torch
    import oracle
    from paper_1904_00182_amd import inputs, nc, workloads
    dev = "cuda:0"
    grid = (32, 16, 32)
    prm = oracle.Params(*grid, alpha=1e3, kappa_f=0.00513)
    F = oracle.cone_filter_matrix(oracle.Mesh(prm), 2.0)
    xo = (F @ inputs.uniform_design(prm.nx * prm.ny * prm.nz, 1) >= 0.5).astype(np.float64)
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    m = oracle.Model(prm, xo)
    so, _ = m.solve_state()
    lo = m.solve_adjoint(so, m.dfds())
    _, go = m.sensitivity(so, lo)
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    p = workloads.problem(grid, 1e3, nc.NC_FP64)
    sol = nc.Solver(p, dev)
    xd = torch.as_tensor(xo, device=dev)
    sol.set_design(xd)
    gg = sol.objective_grad()
    res = {}

    def gpu():
        sol.set_design(xd)
        s = sol.solve_state()
        if sol.last_info["status"] != nc.NC_OK:
            raise RuntimeError("GPU state solve did not converge")
        lam = sol.solve_adjoint(s, gg)
        if sol.last_info["status"] != nc.NC_OK:
            raise RuntimeError("GPU adjoint solve did not converge")
        res.update(s=s, lam=lam, dfdx=sol.sensitivity(s, lam))

    gpu()
    torch.cuda.synchronize()
    reps = 5
    t1 = time.perf_counter()
    for _ in range(reps):
        gpu()
    torch.cuda.synchronize()
    tg = (time.perf_counter() - t1) / reps
    sol.close()
    out = {
        "workload": "cavity 32x16x32 (16384 elements, 92565 dofs), Gr 1e3, U(0,1) design cone-filtered (R=2) "
                    "and thresholded at 0.5 (seed 1), float64 on both sides; state + adjoint + sensitivities",
        "oracle_s": round(wall, 3), "oracle_cores": max(1, int(round(cpu / wall))),
        "oracle_phases_s": {k: round(v, 3) for k, v in m.timing.items()},
        "gpu_fp64_s": round(tg, 5), "ratio": round(wall / tg, 1),
        "gpu_vs_oracle": {
            "state": field_errors(res["s"].cpu(), torch.as_tensor(so), ("u", "v", "w", "P", "T")),
            "adjoint": field_errors(res["lam"].cpu(), torch.as_tensor(lo), (None, None, None, "P", "T")),
            "dfdx": field_errors(res["dfdx"].cpu().reshape(-1, 1), torch.as_tensor(go).reshape(-1, 1), ("dfdx",)),
        },
    }
    log(args, "oracle pair", out)
    return out


def _rel(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / max(float(torch.linalg.vector_norm(b)), 1e-300))


def report(args, path):
    """Extended measurements of the path, written as JSON: operator throughput per grid
    (rotating and cache-resident buffers, float32 and float64), the float64 and mixed
    solves at 128 x 64 x 128 with their difference, a warm-started re-solve after a 1 %
    design perturbation, the oracle's phases beside the GPU solve at small sizes, and the
    serving trace."""
    import numpy as np
    import torch
    from paper_1904_00182_amd import inputs, nc, serve, workloads
    dev = "cuda:0"
    out = {}

    def sync_time(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    # 1. five-field Jacobian apply throughput per grid
    rows = []
    for grid in ((16, 8, 16), (32, 16, 32), (64, 32, 64), (96, 48, 96), (128, 64, 128)):
        p = workloads.problem(grid, 1e4, nc.NC_MIXED)
        sol = nc.Solver(p, dev)
        sol.set_design(workloads.design(grid, "blobs", 2, dev))
        s = sol.solve_state()
        sol.linearize(s)
        N, E = sol.N, sol.E
        for dt, sz in ((torch.float32, 4), (torch.float64, 8)):
            rot = max(2, int(2 * 512e6 / (2 * 5 * N * sz)))
            for tr in (False, True):
                for label, pairs in (("rotating", rot), ("cache_resident", 1)):
                    t = time_apply(sol, torch, dt, tr, 200, pairs)
                    rows.append({"grid": list(grid), "dtype": "f32" if sz == 4 else "f64", "op": "JT w" if tr else "J v",
                                 "buffers": label, "us": round(t * 1e6, 2), "gdofs": round(5 * N / t / 1e9, 2),
                                 "gdofs_pt": round(2 * N / t / 1e9, 2),
                                 "hbm_frac": round((12 * N + 2 * E) * sz / t / 1e9 / HBM_PEAK_GBS, 4)})
        sol.close()
        log(args, "operator", grid, "done")
    out["operator"] = rows

    # 2. float64 and mixed solves at 1M elements, and their difference
    res = {}
    for name in ("cavity128", "cavity128mixed"):
        p, x, cfg = workloads.config(name, dev)
        sol = nc.Solver(p, dev)
        sol.set_design(x)
        g = sol.objective_grad()

        def one():
            s = sol.solve_state()
            i1 = dict(sol.last_info)
            lam = sol.solve_adjoint(s, g)
            i2 = dict(sol.last_info)
            return s, lam, sol.sensitivity(s, lam), i1, i2
        t, (s, lam, dfdx, i1, i2) = sync_time(one)
        res[name] = dict(s=s, lam=lam, dfdx=dfdx)
        out[name] = {"step_s": round(t, 4), "newton_its": i1["newton_its"], "state_krylov_its": i1["krylov_its"],
                     "adjoint_krylov_its": i2["krylov_its"], "adjoint_refinements": i2["refine_its"],
                     "objective": sol.objective(s)}
        if name == "cavity128mixed":
            # warm start after a 1 % perturbation of the design
            gen = inputs.rng(77)
            x2 = torch.clamp(x + 0.01 * torch.as_tensor(gen.uniform(-1, 1, x.numel()), device=dev), 0, 1)
            sol.set_design(x2)
            s_cold = sol.solve_state()
            ic = dict(sol.last_info)

            def warm():
                return sol.solve_state(s0=s)
            tw, _ = sync_time(warm)
            iw = dict(sol.last_info)
            tc, _ = sync_time(lambda: sol.solve_state())
            out["warm_resolve"] = {"perturbation": "x + 0.01 U(-1, 1), clipped to [0, 1]", "cold_state_s": round(tc, 4),
                                   "cold_newton_its": ic["newton_its"], "warm_state_s": round(tw, 4),
                                   "warm_newton_its": iw["newton_its"], "warm_krylov_its": iw["krylov_its"]}
        sol.close()
        log(args, name, out[name])
    a, b = res["cavity128mixed"], res["cavity128"]
    fields = ("u", "v", "w", "P", "T")
    out["mixed_vs_fp64_rel_l2"] = {
        **{f"s_{f}": _rel(a["s"][:, k], b["s"][:, k]) for k, f in enumerate(fields)},
        **{f"lambda_{f}": _rel(a["lam"][:, k], b["lam"][:, k]) for k, f in ((3, "P"), (4, "T"))},
        "dfdx": _rel(a["dfdx"], b["dfdx"])}

    # 3. oracle phases beside the float64 GPU solve at small sizes
    import oracle
    ph = []
    for grid in ((16, 8, 16), (24, 12, 24), (32, 16, 32)):
        nx, ny, nz = grid
        op = oracle.Params(nx, ny, nz, alpha=1e3, kappa_f=0.00513)
        xo = inputs.noise_design(nx * ny * nz, 0)
        t0 = time.perf_counter()
        m = oracle.Model(op, xo)
        so, _ = m.solve_state()
        lo = m.solve_adjoint(so, m.dfds())
        m.sensitivity(so, lo)
        wall = time.perf_counter() - t0
        p = workloads.problem(grid, 1e3, nc.NC_FP64)
        sol = nc.Solver(p, dev)
        sol.set_design(torch.as_tensor(xo, device=dev))
        gg = sol.objective_grad()

        def gpu():
            s = sol.solve_state()
            lam = sol.solve_adjoint(s, gg)
            return sol.sensitivity(s, lam)
        tg, _ = sync_time(gpu, 5)
        sol.close()
        ph.append({"grid": list(grid), "oracle_s": round(wall, 3), "oracle_phases_s": {k: round(v, 3) for k, v in m.timing.items()},
                   "gpu_fp64_s": round(tg, 5)})
        log(args, "oracle", ph[-1])
    out["oracle_vs_gpu"] = ph
    out["host"] = {"cpu_model": _cpu_model(), "cores_available": len(os.sched_getaffinity(0))}

    # 4. serving below saturation (0.8 x capacity), beside the saturated run of the main line
    out["serving_below_saturation"] = serve.run(n=args.report_requests, load=0.8, log=lambda *a: log(args, *a))
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the solver has no multi-GPU path "
              f"(how it would shard is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1904_00182_amd import nc, workloads

    dev = "cuda:0"
    if args.copy_calibration_mb:
        n = args.copy_calibration_mb << 18          # float32 elements
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(args, f"copy calibration: {4 * n} bytes read, {4 * n} bytes written")
        del a, b
    p, x, cfg = workloads.config(args.workload, dev)
    sol = nc.Solver(p, dev)
    N, E = sol.N, sol.E
    sol.set_design(x)
    s = torch.zeros((N, 5), dtype=torch.float64, device=dev)
    lam = torch.zeros_like(s)
    g = sol.objective_grad()
    torch.cuda.synchronize()

    infos = []

    def step():
        # one design iteration's solve path: design chain (filter + RAMP), cold state
        # solve, adjoint, sensitivities
        sol.set_design(x)
        s.zero_()
        sol.solve_state(out=s)
        i_state = dict(sol.last_info)
        sol.solve_adjoint(s, g, out=lam)
        i_adj = dict(sol.last_info)
        if i_state["status"] != nc.NC_OK or i_adj["status"] != nc.NC_OK:
            raise RuntimeError(f"solve did not converge: state {i_state['status']} adjoint {i_adj['status']}")
        dfdx = sol.sensitivity(s, lam)
        infos.append((i_state, i_adj))
        return dfdx

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dfdx = step()
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    i_state, i_adj = infos[-1]
    f_val = sol.objective(s)
    log(args, f"step {t_step * 1e3:.1f} ms  state {i_state}  adjoint {i_adj}  f={f_val:.6e}")
    # the design chain on its own (part of every step above)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        sol.set_design(x)
    torch.cuda.synchronize()
    t_design = (time.perf_counter() - t0) / 20
    mixed_result = (s.clone(), lam.clone(), dfdx.clone())

    # the same steps again with HIP-event timing of every kernel class on the solver's
    # stream: the per-launch durations of the dominant operator kernel inside the solve
    sol.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_step_timed = (time.perf_counter() - t0) / args.steps
    classes = sol.timing()
    sol.timing_bytes = sol.timing(with_bytes=True)
    sol.set_timing(False)
    log(args, "kernel classes (ms, launches) over the instrumented steps:",
        {k: (round(v[0], 2), v[1]) for k, v in classes.items() if v[1]})

    # operator apply throughput and roofline of the dominant kernel (the float32 and
    # float64 five-field Jacobian applies), timed live with HIP events on the solver's stream
    sol.linearize(s)
    mixed = p.precision == nc.NC_MIXED
    wdt = torch.float32 if mixed else torch.float64
    sz = 4 if mixed else 8
    pairs = max(2, int(2 * 512e6 / (2 * 5 * N * sz)))
    t_jv = time_apply(sol, torch, wdt, False, args.apply_iters, pairs)
    t_jv64 = time_apply(sol, torch, torch.float64, False, max(20, args.apply_iters // 2), max(2, pairs // 2))
    t_jtw64 = time_apply(sol, torch, torch.float64, True, max(20, args.apply_iters // 2), max(2, pairs // 2))
    # algorithmic bytes of one apply: read v and write y (5 fields per node), read the
    # linearisation state (P, T per node) and the two element coefficients (k, kappa)
    bytes_jv = (N * (5 + 5 + 2) + E * 2) * sz
    bytes_jv64 = (N * (5 + 5 + 2) + E * 2) * 8
    dofs = 5 * N
    # dominant kernel of the solve: the timed class (each one kernel at one grid size) with
    # the largest summed HIP-event time.  achieved = the class's algorithmic bytes (library
    # accounting: inputs read once, outputs written once) or flops / its summed launch time.
    classes_b = sol.timing_bytes
    dom = max(SINGLE_KERNEL_CLASSES, key=lambda k: classes_b[k][0])
    dom_ms, dom_n, dom_bytes = classes_b[dom]
    t_dom = dom_ms / max(dom_n, 1) * 1e-3
    share = dom_ms / max(1e-9, sum(v[0] for v in classes_b.values()))
    tname = "float" if mixed else "double"
    gbs = dom_bytes / (dom_ms * 1e-3) / 1e9
    hbm = {"achieved_gbs": round(gbs, 1), "peak_gbs": HBM_PEAK_GBS, "frac": round(gbs / HBM_PEAK_GBS, 4),
           "bytes_per_launch": round(dom_bytes / max(dom_n, 1))}
    traffic, valu_insts = measured_counters(dom, tname)
    if dom in FLOPS_PER_ELEM:
        # operator kernels are bound by vector ALU issue: exact flops of the
        # element and node arithmetic, counted on the element code, against the vector peak
        fl = FLOPS_PER_ELEM[dom] * E + FLOPS_PER_NODE[dom] * N
        ach = fl / t_dom / 1e12
        peak = VALU_PEAK_TFLOPS[sz]
        roof = {"bound": "alu", "achieved": round(ach, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(ach / peak, 4), "traffic": traffic,
                "peak_without_packed_fp32": VALU_PEAK_TFLOPS[8], "frac_without_packed_fp32": round(ach / VALU_PEAK_TFLOPS[8], 4),
                "flops_per_launch": fl, "hbm": hbm}
        if valu_insts:
            # VALU issue: one wave64 instruction per SIMD every 4 cycles (1024 SIMDs, 2.4 GHz);
            # the counted instructions of one launch against its live duration
            floor = valu_insts * 4 / (1024 * 2.4e9)
            roof["valu_issue"] = {"instructions_per_launch": round(valu_insts), "floor_us": round(floor * 1e6, 2),
                                  "frac": round(floor / t_dom, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "bytes_per_launch": hbm["bytes_per_launch"]}
    roof.update({"kernel": KERNEL_NAMES[dom].format(t=tname), "class": dom, "launch_us": round(t_dom * 1e6, 2),
                 "launches": dom_n, "share_of_kernel_time": round(share, 3), "timed_step_ms": round(t_step_timed * 1e3, 3)})
    result = {
        "metric": "state+adjoint solve s at 1M elems",
        "value": round(t_step, 5),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"cavity {p.nx}x{p.ny}x{p.nz} Q1 hex ({E} elements, {dofs} dofs at 5/node), Gr "
                        f"{p.alpha:g}, kappa_f {p.kappa_f}, kappa_s {p.kappa_s}, k 1:100, RAMP q=8, unit flux on "
                        f"the centred 0.25x0.25 base patch, seeded U(0,1) design cone-filtered (R=2) and "
                        f"thresholded at 0.5, {'mixed precision (f32 inner, f64 outer)' if mixed else 'float64'}; "
                        f"step = cold Newton state solve + adjoint solve + sensitivities",
            "grid": [p.nx, p.ny, p.nz],
            "elements": E,
            "dofs": dofs,
            "parallelism": "single GPU",
        },
        "roofline": roof,
        "kernel_classes_ms": {k: round(v[0] / args.steps, 3) for k, v in classes.items() if v[1]},
        "operator": {
            "jv_working_precision_us": round(t_jv * 1e6, 2),
            "jv_working_precision_hbm_frac": round(bytes_jv / t_jv / 1e9 / HBM_PEAK_GBS, 4),
            "gdofs_jv_working_precision": round(dofs / t_jv / 1e9, 3),
            "gdofs_jv_f64": round(dofs / t_jv64 / 1e9, 3),
            "gdofs_jtw_f64": round(dofs / t_jtw64 / 1e9, 3),
            "gdofs_pt_only_jv_working_precision": round(2 * N / t_jv / 1e9, 3),
            "jv_f64_us": round(t_jv64 * 1e6, 2),
            "jtw_f64_us": round(t_jtw64 * 1e6, 2),
            "jv_f64_hbm_frac": round(bytes_jv64 / t_jv64 / 1e9 / HBM_PEAK_GBS, 4),
        },
        "solve": {
            "state_status": nc_status(i_state["status"]), "adjoint_status": nc_status(i_adj["status"]),
            "newton_its": i_state["newton_its"], "state_krylov_its": i_state["krylov_its"],
            "state_krylov_per_newton_step": i_state["hist_krylov"],
            "adjoint_krylov_its": i_adj["krylov_its"], "adjoint_refinements": i_adj["refine_its"],
            "levels": i_state["levels"], "state_s": round(i_state["t_total"], 4),
            "state_setup_s": round(i_state["t_setup"], 5),
            "adjoint_s": round(i_adj["t_total"], 4), "set_design_ms": round(t_design * 1e3, 3),
            "objective": f_val,
            "state_residual_per_field": {"initial": i_state["res0"], "final": i_state["res"]},
        },
    }
    sol.close()
    del sol
    torch.cuda.empty_cache()
    result["pde_filter"] = pde_filter_timing(args)
    if not args.no_design_loop:
        result["design_loop"] = design_loop_timing(args)
    if not args.no_ns:
        result["navier_stokes"] = ns_timing(args)
    if args.paper_runs > 0:
        result["paper_optimisation"] = paper_runs(args)
    if mixed and not args.no_fp64_leg:
        result["fp64_baseline"] = fp64_leg(args, mixed_result)
        result["fp64_baseline"]["mixed_speedup"] = round(result["fp64_baseline"]["ms_per_step"] / (t_step * 1e3), 3)
    if not args.no_serving:
        from paper_1904_00182_amd import serve
        result["serving"] = serve.run(n=args.serving_requests, load=args.serving_load, log=lambda *a: log(args, *a))
    if not args.no_oracle_pair:
        result["oracle_pair"] = oracle_pair(args)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, E)
    if args.report:
        report(args, args.report)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
