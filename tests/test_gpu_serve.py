"""Serving loop: admission under a memory budget and continuous batching.
Each request's result must equal the same request run alone (bit-identical),
whatever it was batched with and whenever it was admitted."""
import numpy as np
import pytest

from gpu_common import gpu_context, say

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone(xs_default):
    say("test_served_results_equal_alone")
    from paper_2103_09642_amd import edupic
    from paper_2103_09642_amd.serve import Request, Server, case_for, latency_summary
    ctx = gpu_context()
    ctx.set_xsec(xs_default)
    ctx.set_option(edupic.OPT_MODE, 1)
    ctx.set_option(edupic.OPT_SORT_EVERY, 50)
    items = [(0, 3, 1), (0, 17, 2), (1, 5, 3), (2, 40, 1), (2, 9, 2), (4, 61, 1)]  # (arrival iteration, case k, cycles)
    reqs = [Request(i, float(t), case_for({"kind": "batch", "case_k": k}, n_scale=0.02), cyc)
            for i, (t, k, cyc) in enumerate(items)]
    sizes = [ctx.case_bytes(r.case) for r in reqs]
    budget = 2 * max(sizes)  # at most two resident at once
    srv = Server(ctx, budget, clock=lambda: float(srv.iterations))
    done = srv.run(reqs, virtual=True)
    assert len(done) == len(reqs)
    assert max(r.t_admit - r.t_arrival for r in done) > 0, "the budget never made a request wait"
    summ = latency_summary(done)
    assert summ["n"] == len(reqs) and summ["p99_s"] >= summ["p50_s"] > 0
    for r in done:
        g = ctx.create_case(r.case)
        g.advance(r.cycles)
        k = g.counts()
        ne, ni = g.density()
        g.destroy()
        assert k == r.result["counts"], f"request {r.rid}: counters"
        assert np.array_equal(ne, r.result["ne"]) and np.array_equal(ni, r.result["ni"]), f"request {r.rid}: densities"
    ctx.set_option(edupic.OPT_MODE, 0)
    ctx.set_option(edupic.OPT_SORT_EVERY, 100)
