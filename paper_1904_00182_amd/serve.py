"""Continuous-batching request server for state + adjoint solves on one GPU.

Requests (a grid, a Grashof number, a heat-flux magnitude, a design seed and a
precision) arrive over time.  The scheduler admits a waiting request as soon as a slot
is free and its device footprint (the solver workspace from nc_workspace_bytes plus its
state, adjoint, design and gradient arrays) fits under the memory cap; admitted
requests run concurrently, each on its own HIP stream and host worker thread, so their
kernels overlap on the device, and their state stays resident in HBM between the state
solve and the adjoint solve.  Requests that do not fit wait in arrival order; a request
that can never fit is rejected.  Latency is measured from arrival to completion (the
moment its results are on the device and its stream has drained).

Each slot keeps its solver contexts, one per (grid, precision), and serves a new
request on a kept context through nc_set_problem: no context is created or destroyed
per request (destroying one frees pinned host memory, which waits for the whole
device).  A request whose state or adjoint solve does not converge is recorded as
such and counted neither as completed nor in the latency percentiles.

The scheduling core (`Scheduler`) is independent of the GPU: it drives any backend with
`footprint(req)` and `run(req, slot)` methods, which lets the CPU test-suite exercise it
with a fake backend.
"""

import heapq
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    id: int
    arrival: float
    grid: tuple
    gr: float
    q_h: float
    design_seed: int
    precision: int = 0
    # filled by the scheduler
    admit: float = None
    finish: float = None
    status: str = "pending"
    result: dict = field(default_factory=dict)

    @property
    def latency(self):
        return None if self.finish is None else self.finish - self.arrival


class Scheduler:
    """Admission by memory footprint and free slots, FIFO among waiting requests,
    concurrent execution on `slots` workers."""

    def __init__(self, backend, slots=4, mem_cap=8 << 30, clock=time.perf_counter, sleep=time.sleep):
        self.backend = backend
        self.slots = slots
        self.mem_cap = mem_cap
        self.clock = clock
        self.sleep = sleep
        self.lock = threading.Condition()
        self.in_use = 0
        self.active = 0
        self.free_slots = list(range(slots))
        self.log = []

    def _worker(self, req, slot, fp):
        try:
            req.result = self.backend.run(req, slot) or {}
            req.status = req.result.pop("status", "done")
        except Exception as e:  # the failure is recorded on the request
            req.status = f"failed: {e}"
        with self.lock:
            req.finish = self.clock() - self.t0
            self.in_use -= fp
            self.active -= 1
            self.free_slots.append(slot)
            self.log.append(("finish", req.id, req.finish))
            self.lock.notify_all()

    def serve(self, requests):
        """Run every request; arrival times are seconds after the start.  Returns the
        requests (with admit / finish times and status)."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.id))
        waiting = []
        threads = []
        self.t0 = self.clock()
        i = 0
        while i < len(pending) or waiting or self.active:
            now = self.clock() - self.t0
            while i < len(pending) and pending[i].arrival <= now:
                r = pending[i]
                fp = self.backend.footprint(r)
                if fp > self.mem_cap:
                    r.status = "rejected: footprint above the memory cap"
                    r.finish = now
                    self.log.append(("reject", r.id, now))
                else:
                    waiting.append((r, fp))
                    self.log.append(("arrive", r.id, now))
                i += 1
            with self.lock:
                # FIFO admission: the head of the queue goes first when it fits
                while waiting and self.free_slots and self.in_use + waiting[0][1] <= self.mem_cap:
                    r, fp = waiting.pop(0)
                    slot = self.free_slots.pop(0)
                    self.in_use += fp
                    self.active += 1
                    r.admit = self.clock() - self.t0
                    self.log.append(("admit", r.id, r.admit, slot))
                    t = threading.Thread(target=self._worker, args=(r, slot, fp), daemon=True)
                    threads.append(t)
                    t.start()
                if i < len(pending):
                    wait = max(0.0, pending[i].arrival - (self.clock() - self.t0))
                    if wait > 0:
                        self.lock.wait(timeout=min(wait, 0.05))
                elif waiting or self.active:
                    self.lock.wait(timeout=0.05)
        for t in threads:
            t.join()
        return requests


def summarize(requests, wall):
    done = [r for r in requests if r.status == "done"]
    lat = np.array([r.latency for r in done]) if done else np.zeros(1)
    return {
        "requests": len(requests),
        "completed": len(done),
        "rejected": sum(1 for r in requests if r.status.startswith("rejected")),
        "failed": sum(1 for r in requests if r.status.startswith("failed")),
        "not_converged": sum(1 for r in requests if r.status == "not converged"),
        "p50_s": float(np.percentile(lat, 50)),
        "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()),
        "solves_per_s": len(done) / wall if wall > 0 else 0.0,
        "wall_s": wall,
    }


class GPUBackend:
    """Runs one request as: design generation, state solve, adjoint solve and
    sensitivities on its slot's stream, keeping the arrays resident until done.
    force_precision overrides every request's precision (the plain float64 baseline)."""

    def __init__(self, device="cuda:0", slots=4, keep_results=False, force_precision=None):
        import torch
        from . import nc
        self.torch = torch
        self.nc = nc
        self.device = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(slots)]
        self.keep = keep_results
        self.force = force_precision
        self.pools = [dict() for _ in range(slots)]   # per slot: (grid, precision) -> Solver

    def precision(self, req):
        return req.precision if self.force is None else self.force

    def problem(self, req):
        from . import workloads
        return workloads.problem(req.grid, req.gr, precision=self.precision(req), q_h=req.q_h)

    def solver(self, req, slot):
        """The slot's kept context for the request's layout, set to its parameters."""
        p = self.problem(req)
        key = (tuple(req.grid), self.precision(req))
        sol = self.pools[slot].get(key)
        if sol is None:
            sol = self.nc.Solver(p, self.device, stream=self.streams[slot])
            self.pools[slot][key] = sol
        else:
            sol.set_problem(p)
        return sol

    def footprint(self, req):
        nx, ny, nz = req.grid
        N = (nx + 1) * (ny + 1) * (nz + 1)
        E = nx * ny * nz
        return self.nc.workspace_bytes(self.problem(req)) + 256 + 3 * 5 * N * 8 + 3 * E * 8

    def run(self, req, slot):
        torch, nc = self.torch, self.nc
        from . import workloads
        st = self.streams[slot]
        with torch.cuda.stream(st):
            x = workloads.design(req.grid, "blobs", req.design_seed, self.device)
            sol = self.solver(req, slot)
            sol.set_design(x)
            s = sol.solve_state()
            i_state = dict(sol.last_info)
            g = sol.objective_grad()
            lam = sol.solve_adjoint(s, g)
            i_adj = dict(sol.last_info)
            dfdx = sol.sensitivity(s, lam)
            f = sol.objective(s)
            st.synchronize()
            ok = i_state["status"] == nc.NC_OK and i_adj["status"] == nc.NC_OK
            out = {"f": f, "state": i_state, "adjoint": i_adj, "status": "done" if ok else "not converged"}
            if self.keep:
                out.update(s=s.cpu(), lam=lam.cpu(), dfdx=dfdx.cpu())
            return out

    def close(self):
        for pool in self.pools:
            for sol in pool.values():
                sol.close()
            pool.clear()


def make_requests(n, rate, seed=4, grids=((16, 8, 16), (32, 16, 32), (64, 32, 64), (96, 48, 96)),
                  grs=(1e3, 1e4), mixed_fraction=0.5):
    """The serving workload: Poisson arrivals at `rate`/s, grid and Gr drawn per request,
    q_h ~ U(0.5, 2), design seed 1000 + r; precision alternates FP64 / mixed by a draw."""
    from . import inputs
    draws = inputs.request_stream(n, rate, seed, grids, grs)
    g = inputs.rng(seed + 1)
    out = []
    for d in draws:
        prec = 1 if g.uniform() < mixed_fraction else 0
        out.append(Request(d["id"], d["arrival"], d["grid"], d["gr"], d["q_h"], d["design_seed"], prec))
    return out


def _warm(be, slots):
    """Creates every slot's contexts for the mix's grids and precisions (one small solve
    each), so that measured requests find them kept."""
    for slot in range(slots):
        for i, gsz in enumerate(((16, 8, 16), (32, 16, 32), (64, 32, 64), (96, 48, 96))):
            for prec in (0, 1):
                be.run(Request(-1 - i, 0.0, gsz, 1e3, 1.0, 999, prec), slot)


def run(n=256, rate=None, load=1.5, slots=4, mem_cap=16 << 30, seed=4, device="cuda:0", log=print):
    """Serve n requests of the mixed-size, mixed-precision trace with continuous batching
    (`slots` concurrent requests, each on its own stream) and, as the baseline, the same
    trace served FIFO one at a time with the plain float64 solve.  With rate=None the
    arrival rate is `load` x the measured one-at-a-time capacity of the mix (load > 1:
    saturation, where throughput can differ).  Returns both summaries."""
    import torch
    be = GPUBackend(device, slots)
    base = GPUBackend(device, 1, force_precision=0)
    _warm(be, slots)
    _warm(base, 1)
    torch.cuda.synchronize()
    probe = make_requests(24, 1e9, seed + 7)
    t0 = time.perf_counter()
    for r in probe:
        be.run(r, 0)
    cap = len(probe) / (time.perf_counter() - t0)
    if rate is None:
        rate = load * cap
    log(f"one-at-a-time capacity {cap:.1f} solves/s -> arrival rate {rate:.1f}/s")
    res = {"arrival_rate_per_s": round(rate, 2), "one_at_a_time_capacity_per_s": round(cap, 2), "requests": n,
           "slots": slots, "mem_cap_bytes": mem_cap,
           "trace": "Poisson arrivals; grids 16x8x16 .. 96x48x96, Gr 1e3 / 1e4, q_h ~ U(0.5, 2), blob design "
                    "seed 1000 + r, float64 or mixed with probability 1/2 (the baseline solves all in float64)"}
    for label, backend, sl in (("continuous", be, slots), ("fifo_serial_fp64", base, 1)):
        reqs = make_requests(n, rate, seed)
        sch = Scheduler(backend, slots=sl, mem_cap=mem_cap)
        t0 = time.perf_counter()
        sch.serve(reqs)
        wall = time.perf_counter() - t0
        s = summarize(reqs, wall)
        for prec, nm in ((0, "fp64"), (1, "mixed")):
            lat = [r.latency for r in reqs if r.status == "done" and r.precision == prec]
            if lat and label == "continuous":
                s[f"p50_s_{nm}"] = float(np.percentile(lat, 50))
                s[f"p99_s_{nm}"] = float(np.percentile(lat, 99))
        res[label] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in s.items()}
        log(label, res[label])
    be.close()
    base.close()
    return res


if __name__ == "__main__":
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=None)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--mem-cap-gb", type=float, default=16.0)
    a = ap.parse_args()
    out = run(a.requests, a.rate, a.slots, int(a.mem_cap_gb * (1 << 30)), log=lambda *x: print(*x, file=sys.stderr))
    print(json.dumps(out))
