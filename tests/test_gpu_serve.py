"""Serving loop: admission under a memory budget, continuous batching in
fixed step windows, capacity growth and per-request failure.  Each request's
result must equal the same request run alone (bit-identical), whatever it
was batched with, whenever it was admitted and however often it was moved
to a larger arena."""
import numpy as np
import pytest

from gpu_common import by_uid, gpu_context, say
from paper_2103_09642_amd.workloads import base_case, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(xs_default):
    from paper_2103_09642_amd import edupic
    c = gpu_context()
    c.set_xsec(xs_default)
    c.set_option(edupic.OPT_MODE, 1)
    c.set_option(edupic.OPT_SORT_EVERY, 50)
    yield c
    c.set_option(edupic.OPT_MODE, 0)
    c.set_option(edupic.OPT_SORT_EVERY, 100)


def _alone(ctx, r):
    c = dict(r.case)
    g = ctx.create_case(c)
    g.advance(r.cycles)
    k = g.counts()
    ne, ni = g.density()
    g.destroy()
    return k, ne, ni


def test_served_results_equal_alone(ctx):
    """Six batched-set requests (2% of their particles) through a budget that
    holds at most two, in windows of 1500 steps: every result equals the
    request run alone, and the budget made requests wait."""
    say("test_served_results_equal_alone")
    from paper_2103_09642_amd.serve import Request, Server, case_for, latency_summary
    items = [(0, 3, 1), (0, 17, 2), (1, 5, 3), (2, 40, 1), (2, 9, 2), (4, 61, 1)]  # (arrival iteration, case k, cycles)
    reqs = [Request(i, float(t), case_for({"kind": "batch", "case_k": k}, n_scale=0.02), cyc)
            for i, (t, k, cyc) in enumerate(items)]
    sizes = [ctx.case_bytes(r.case) for r in reqs]
    budget = 2 * max(sizes) + (max(sizes) // 2)  # about two resident at once, room to grow one
    srv = Server(ctx, budget, window=1500, clock=lambda: float(srv.iterations))
    done = srv.run(reqs, virtual=True)
    assert len(done) == len(reqs) and not srv.failed
    assert max(r.t_admit - r.t_arrival for r in done) > 0, "the budget never made a request wait"
    summ = latency_summary(done)
    assert summ["n"] == len(reqs) and summ["p99_s"] >= summ["p50_s"] > 0
    for r in done:
        k, ne, ni = _alone(ctx, r)
        got = dict(r.result["counts"])
        assert k == got, f"request {r.rid}: counters"
        assert np.array_equal(ne, r.result["ne"]) and np.array_equal(ni, r.result["ni"]), f"request {r.rid}"


def test_resize_continues_bit_for_bit(ctx):
    """A case moved to an arena with twice (then again other) capacities
    mid-run, with collisions, births and sorts going on, ends exactly where
    the same case with ample room from the start ends."""
    say("test_resize_continues_bit_for_bit")
    c = base_case(n_init_e=0, n_init_i=0, pressure_pa=40.0, weight=1e6, ion_subcycle=5, cap_e=20_000,
                  cap_i=20_000, flags=["allow_unstable", "density", "eepf"])
    st = random_state(9000, 9000, c["gap_m"], seed=91, te_ev=4.0, hot_frac=0.3, hot_ev=90.0)
    ref = ctx.create_case(dict(c, cap_e=80_000, cap_i=80_000))
    g = ctx.create_case(c)
    for x in (ref, g):
        x.set_state(0, st["e"], 0)
        x.set_state(1, st["i"], 0)
    ref.advance_steps(330)
    g.advance_steps(123)
    g.resize(40_192, 40_192)
    g.advance_steps(100)
    g.resize(60_160, 0)
    g.advance_steps(107)
    assert g.capacity() == (60_160, 40_192)
    assert ref.counts() == g.counts()
    for sp in (0, 1):
        a, b = by_uid(ref.get_state(sp)), by_uid(g.get_state(sp))
        for k in ("uid", "x", "vx", "vy", "vz"):
            assert np.array_equal(a[k], b[k]), (sp, k)
    for a, b in zip(ref.deposit(), g.deposit()):
        assert np.array_equal(a, b)
    for a, b in zip(ref.density(), g.density()):
        assert np.array_equal(a, b)
    assert np.array_equal(ref.eepf()[1], g.eepf()[1])
    ref.destroy()
    g.destroy()


def test_overflow_fails_only_that_request(ctx):
    """A request seeded at its full capacity with no room to grow (capacity
    limit = its capacity) overflows at its first ionization: it alone fails,
    the other requests of the mix complete with their alone results, and a
    request that grows past its first capacity is resized and completes."""
    say("test_overflow_fails_only_that_request")
    from paper_2103_09642_amd.serve import Request, Server, case_for
    full = case_for({"kind": "batch", "case_k": 47}, n_scale=0.02)
    n = full["n_init_e"] // 256 * 256
    full = dict(full, n_init_e=n, n_init_i=n, cap_e=n, cap_i=n)
    grow = case_for({"kind": "batch", "case_k": 47}, n_scale=0.02)
    grow = dict(grow, cap_e=(grow["n_init_e"] + 4095) // 256 * 256, cap_i=(grow["n_init_i"] + 4095) // 256 * 256)
    reqs = [Request(0, 0.0, case_for({"kind": "batch", "case_k": 12}, n_scale=0.02), 1),
            Request(1, 0.0, full, 2, cap_limit=n),
            Request(2, 1.0, grow, 2),
            Request(3, 1.0, case_for({"kind": "batch", "case_k": 33}, n_scale=0.02), 1)]
    srv = Server(ctx, 1 << 40, window=400, clock=lambda: float(srv.iterations))
    done = srv.run(reqs, virtual=True)
    assert [r.rid for r in srv.failed] == [1] and srv.failed[0].failed == "capacity"
    assert srv.failed[0].result["counts"]["dropped"] > 0
    assert sorted(r.rid for r in done) == [0, 2, 3]
    assert reqs[2].resizes >= 1
    for r in done:
        k, ne, ni = _alone(ctx, r)
        assert k == r.result["counts"], f"request {r.rid}: counters"
        assert np.array_equal(ne, r.result["ne"]) and np.array_equal(ni, r.result["ni"])
