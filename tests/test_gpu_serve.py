"""Serving on the GPU: requests of different grids and precisions run concurrently on
their own streams; every result is bitwise identical to the same request run alone."""

import numpy as np
import pytest
import torch

from paper_1904_00182_amd.serve import GPUBackend, Request, Scheduler, summarize

pytestmark = pytest.mark.gpu


def test_alone_vs_in_the_mix_bitwise():
    reqs = [Request(0, 0.0, (16, 8, 16), 1e3, 1.3, 1000, 0), Request(1, 0.0, (32, 16, 32), 1e4, 0.7, 1001, 1),
            Request(2, 0.0, (24, 12, 24), 1e3, 1.9, 1002, 0), Request(3, 0.0, (16, 8, 16), 1e4, 0.5, 1003, 1),
            Request(4, 0.0, (32, 16, 32), 1e3, 1.1, 1004, 0), Request(5, 0.0, (8, 4, 8), 1e4, 2.0, 1005, 1)]
    be = GPUBackend("cuda:0", slots=4, keep_results=True)
    alone = {}
    for r in reqs:
        rr = Request(r.id, 0.0, r.grid, r.gr, r.q_h, r.design_seed, r.precision)
        alone[r.id] = be.run(rr, 0)
    mix = [Request(r.id, 0.0, r.grid, r.gr, r.q_h, r.design_seed, r.precision) for r in reqs]
    sch = Scheduler(be, slots=4, mem_cap=8 << 30)
    sch.serve(mix)
    assert all(r.status == "done" for r in mix), [r.status for r in mix]
    # several requests were on the device at the same time
    admits = sorted((r.admit, r.finish) for r in mix)
    assert any(a2 < f1 for (a1, f1), (a2, f2) in zip(admits, admits[1:]))
    for r in mix:
        a = alone[r.id]
        for key in ("s", "lam", "dfdx"):
            assert torch.equal(a[key], r.result[key]), (r.id, key)
        assert a["f"] == r.result["f"]


def test_memory_cap_rejects_and_serialises():
    be = GPUBackend("cuda:0", slots=4)
    small = Request(0, 0.0, (8, 4, 8), 1e3, 1.0, 1000, 0)
    big = Request(1, 0.0, (64, 32, 64), 1e3, 1.0, 1001, 0)
    cap = be.footprint(small) * 2 + 1
    reqs = [small, big, Request(2, 0.0, (8, 4, 8), 1e3, 1.0, 1002, 0), Request(3, 0.0, (8, 4, 8), 1e3, 1.0, 1003, 0)]
    Scheduler(be, slots=4, mem_cap=cap).serve(reqs)
    assert reqs[1].status.startswith("rejected")
    assert all(r.status == "done" for r in (reqs[0], reqs[2], reqs[3]))
    s = summarize(reqs, max(r.finish for r in reqs))
    assert s["completed"] == 3 and s["rejected"] == 1
