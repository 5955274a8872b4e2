#!/usr/bin/env python3
"""Benchmark of the natural-convection state + adjoint solve on one MI355X.

One step = the whole hot path for one design on the 128 x 64 x 128 cavity (1,048,576
elements, 5,408,325 dofs), Gr = 1e4, filtered-noise 0/1 design, mixed precision:
cold-start Newton state solve (float64 residual and update, float32 FGMRES + multigrid
inner solves), the objective gradient, the adjoint solve (float32 inner, float64
refinement) and the sensitivities through RAMP and the filter.  Inputs are resident in
HBM before the timed region.

Printed: one JSON line with the step time (the metric is "state+adjoint solve s at 1M
elems", lower is better), the live HIP-event timing of the dominant operator kernel
against the HBM roofline, operator GDoF/s, and the float64 CPU oracle timed on a small
sample of the same workload on this host.
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

# kernel symbol of each timed class (tile template arguments elided)
KERNEL_NAMES = {
    "jv": "zmarch_kernel<JvOp<{t},2,0>,..,1> (Krylov operator: (P, T) block of J)",
    "jtw": "zmarch_kernel<JtwOp<{t},2,0>,..,1> (Krylov operator: (P, T) block of J^T)",
    "smooth": "zmarch_kernel<JvOp<{t},2,2>,..,1> (finest-grid block-Jacobi sweep)",
    "smooth_T": "zmarch_kernel<JtwOp<{t},2,2>,..,1> (finest-grid transposed block-Jacobi sweep)",
    "smooth_coarse": "zmarch_kernel<JvOp/JtwOp<{t},2,2>,..,0> (block-Jacobi sweeps, coarse levels)",
    "pt_residual": "zmarch_kernel<JvOp/JtwOp<{t},2,1>,..> (multigrid residual)",
    "mdot": "mdot_kernel<{t}> (FGMRES multi-dot)",
    "maxpy": "maxpy_kernel<{t}> (FGMRES multi-axpy)",
    "transfer": "restrict/prolong/diag_scale kernels (grid transfers)",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cavity128mixed")
    ap.add_argument("--apply-iters", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-grid", default="20,10,20")
    ap.add_argument("--quiet", action="store_true")
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
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU execution is not part of "
              f"this build", file=sys.stderr)
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
        s.zero_()
        sol.solve_state(out=s)
        i_state = dict(sol.last_info)
        sol.solve_adjoint(s, g, out=lam)
        i_adj = dict(sol.last_info)
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
    # dominant kernel class of the solve (by summed HIP-event time) and its roofline:
    # achieved = the class's algorithmic bytes (library accounting: inputs read once,
    # outputs written once) / its summed launch time
    classes_b = sol.timing_bytes
    dom = max(classes_b, key=lambda k: classes_b[k][0])
    dom_ms, dom_n, dom_bytes = classes_b[dom]
    t_dom = dom_ms / max(dom_n, 1) * 1e-3
    ach = dom_bytes / (dom_ms * 1e-3) / 1e9
    share = dom_ms / max(1e-9, sum(v[0] for v in classes_b.values()))
    roof = {
        "kernel": KERNEL_NAMES.get(dom, dom).format(t="float" if mixed else "double"),
        "bound": "hbm",
        "achieved": round(ach, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(ach / HBM_PEAK_GBS, 4),
        "traffic": None,
        "class": dom,
        "launch_us": round(t_dom * 1e6, 2),
        "launches": dom_n,
        "bytes_per_launch": round(dom_bytes / max(dom_n, 1)),
        "share_of_kernel_time": round(share, 3),
        "timed_step_ms": round(t_step_timed * 1e3, 3),
    }
    if dom in FLOPS_PER_ELEM:
        # arithmetic side of the operator kernels: exact flops of the element and node
        # arithmetic (counted on the element code itself) against the vector peak
        fl = FLOPS_PER_ELEM[dom] * E + FLOPS_PER_NODE[dom] * N
        peak = VALU_PEAK_TFLOPS[sz]
        roof["alu"] = {"achieved_tflops": round(fl / t_dom / 1e12, 2), "peak_tflops": peak,
                       "frac": round(fl / t_dom / 1e12 / peak, 4), "flops_per_launch": fl,
                       "flops_per_byte": round(fl / (dom_bytes / max(dom_n, 1)), 2)}
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
            "newton_its": i_state["newton_its"], "state_krylov_its": i_state["krylov_its"],
            "adjoint_krylov_its": i_adj["krylov_its"], "adjoint_refinements": i_adj["refine_its"],
            "levels": i_state["levels"], "state_s": round(i_state["t_total"], 4),
            "adjoint_s": round(i_adj["t_total"], 4), "objective": f_val,
        },
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, E)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
