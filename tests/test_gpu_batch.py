"""Batched execution: several cases advanced by one call, every launch
serving all of them.  A case's result must not depend on what it is batched
with: bit-identical to the same case advanced alone (integer deposits,
random numbers keyed by particle identity and step, per-case sort schedule).
"""
import numpy as np
import pytest

from gpu_common import by_uid, compare_states, gpu_context, say
from paper_2103_09642_amd.workloads import base_case, random_state

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(xs_default):
    c = gpu_context()
    c.set_xsec(xs_default)
    return c


def _mix():
    """Four different cases: grids, subcycling, pressures, sizes, gaps."""
    specs = [
        dict(n_grid=400, ion_subcycle=20, pressure_pa=20.0, gap_m=0.025, n=30_000, seed=21),
        dict(n_grid=173, ion_subcycle=5, pressure_pa=60.0, gap_m=0.015, n=8_000, seed=22),
        dict(n_grid=1000, ion_subcycle=20, pressure_pa=10.0, gap_m=0.04, n=50_000, seed=23),
        dict(n_grid=2, ion_subcycle=3, pressure_pa=5.0, gap_m=0.02, n=1_000, seed=24),
    ]
    out = []
    for sp in specs:
        n = sp.pop("n")
        seed = sp.pop("seed")
        c = base_case(n_init_e=0, n_init_i=0, weight=1e5, flags=["allow_unstable"], cap_e=4 * n, cap_i=4 * n,
                      seed=seed, **sp)
        st = random_state(n, n, c["gap_m"], seed=seed, te_ev=3.0, hot_frac=0.2, hot_ev=80.0)
        out.append((c, st))
    return out


def _make(ctx, c, st, step0):
    g = ctx.create_case(c)
    g.set_state(0, st["e"], step0)
    g.set_state(1, st["i"], step0)
    return g


def _result(g):
    return by_uid(g.get_state(0)), by_uid(g.get_state(1)), g.deposit(), g.counts()


def _same(a, b, label):
    for sp in (0, 1):
        for k in ("uid", "x", "vx", "vy", "vz"):
            assert np.array_equal(a[sp][k], b[sp][k]), f"{label}: species {sp} {k}"
    assert np.array_equal(a[2][0], b[2][0]) and np.array_equal(a[2][1], b[2][1]), f"{label}: deposit"
    assert a[3] == b[3], f"{label}: counters"


@pytest.mark.parametrize("groups", [1, 2, 4])
@pytest.mark.parametrize("mode", [0, 1], ids=["plain", "graph"])
def test_batch_equals_alone(ctx, mode, groups):
    """Different step counts (the batch shrinks as cases finish) and
    different starting steps (different ion-step and sort phases); in one
    lockstep group, and split into two or four groups on streams of their
    own."""
    say(f"test_batch_equals_alone mode={mode} groups={groups}")
    from paper_2103_09642_amd import edupic
    ctx.set_option(edupic.OPT_MODE, mode)
    ctx.set_option(edupic.OPT_SORT_EVERY, 10)
    ctx.set_option(edupic.OPT_GROUPS, groups)
    mix = _mix()
    steps = [700, 433, 700, 120]
    starts = [0, 3, 17, 5]
    alone = []
    for (c, st), n, s0 in zip(mix, steps, starts):
        g = _make(ctx, c, st, s0)
        g.advance_steps(n)
        alone.append(_result(g))
        g.destroy()
    gs = [_make(ctx, c, st, s0) for (c, st), s0 in zip(mix, starts)]
    ctx.advance_steps(gs, steps)
    for k, g in enumerate(gs):
        r = _result(g)
        assert r[3]["step"] == starts[k] + steps[k]
        _same(alone[k], r, f"case {k}")
        g.destroy()
    ctx.set_option(edupic.OPT_MODE, 0)
    ctx.set_option(edupic.OPT_SORT_EVERY, 100)
    ctx.set_option(edupic.OPT_GROUPS, 1)
    for bad in (0, 5):
        with pytest.raises(edupic.EdpError):
            ctx.set_option(edupic.OPT_GROUPS, bad)


def test_chunk_shares_change_nothing(ctx):
    """A case with more chunks than the chip has resident particle
    workgroups (so its workgroups span several dispatch layers): its result
    is bit-identical whatever weighting of the workgroups' chunk shares
    (EDP_OPT_PART_SKEW), workgroups per CU and collision pre-test bound
    (EDP_OPT_PRETEST: P* over the table, or by energy block) the launches
    use."""
    from paper_2103_09642_amd import edupic
    say("test_chunk_shares_change_nothing")
    n = 400_000
    c = base_case(n_init_e=0, n_init_i=0, weight=1e3, n_grid=1000, pressure_pa=30.0, flags=["allow_unstable"],
                  cap_e=2 * n, cap_i=2 * n, seed=31)
    st = random_state(n, n, c["gap_m"], seed=31, te_ev=3.0, hot_frac=0.2, hot_ev=80.0)
    ctx.set_option(edupic.OPT_SORT_EVERY, 10)
    res = []
    for skew, wg, pre in ((0, 0, 1), (-1, 0, 0), (900, 0, 2), (450, 3, 2)):
        ctx.set_option(edupic.OPT_PART_SKEW, skew)
        ctx.set_option(edupic.OPT_PART_WG_PER_CU, wg)
        ctx.set_option(edupic.OPT_PRETEST, pre)
        g = _make(ctx, c, st, 7)
        g.advance_steps(45)
        res.append(_result(g))
        g.destroy()
    ctx.set_option(edupic.OPT_PART_SKEW, -1)
    ctx.set_option(edupic.OPT_PART_WG_PER_CU, 0)
    ctx.set_option(edupic.OPT_PRETEST, 0)
    ctx.set_option(edupic.OPT_SORT_EVERY, 100)
    for k in range(1, len(res)):
        _same(res[0], res[k], f"schedule {k}")
    assert res[0][3]["ioniz"] > 0 and res[0][3]["coll_e"] > 0
    for bad in (-2, 901):
        with pytest.raises(edupic.EdpError):
            ctx.set_option(edupic.OPT_PART_SKEW, bad)
    for bad in (-1, 3):
        with pytest.raises(edupic.EdpError):
            ctx.set_option(edupic.OPT_PRETEST, bad)


def test_batch_matches_oracle(ctx, xs_default, orc):
    """Three cases advanced together for 40 steps against three oracle runs:
    counters exact, states to the one-step bar (with the flux solve's field
    kick as the velocity floor)."""
    say("test_batch_matches_oracle")
    mix = _mix()[:3]
    gs, os_ = [], []
    for c, st in mix:
        gs.append(_make(ctx, c, st, 0))
        o = orc.Oracle(c, xs_default)
        o.set_state(0, st["e"], 0)
        o.set_state(1, st["i"], 0)
        os_.append(o)
    ctx.advance_steps(gs, [40, 40, 40])
    for (c, _), g, o in zip(mix, gs, os_):
        o.step(40)
        cg, co = g.counts(), o.counts()
        for k in ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz"):
            assert cg[k] == co[k], k
        for sp in (0, 1):
            compare_states(g.get_state(sp), o.get_state(sp), 1e-9, f"ng={c['n_grid']} sp{sp}")
        g.destroy()


def test_groups_with_empty_cases(ctx):
    """Four groups over a batch of empty cases (no expected work, so the
    split goes by case count) and one populated case: every case reaches its
    step, and the populated one equals itself advanced alone."""
    say("test_groups_with_empty_cases")
    from paper_2103_09642_amd import edupic
    c, st = _mix()[1]
    g = _make(ctx, c, st, 0)
    g.advance_steps(60)
    alone = _result(g)
    g.destroy()
    empty = {"x": np.zeros(0), "vx": np.zeros(0), "vy": np.zeros(0), "vz": np.zeros(0),
             "uid": np.zeros(0, dtype=np.uint64)}
    gs = [_make(ctx, c, {"e": empty, "i": empty}, 0) for _ in range(4)] + [_make(ctx, c, st, 0)]
    ctx.set_option(edupic.OPT_GROUPS, 4)
    try:
        ctx.advance_steps(gs, [60] * len(gs))
        assert all(x.counts()["step"] == 60 for x in gs)
        assert all(x.counts()["n_e"] == 0 for x in gs[:4])
        _same(alone, _result(gs[4]), "populated case")
    finally:
        ctx.set_option(edupic.OPT_GROUPS, 2)
        for x in gs:
            x.destroy()


def test_batch_rejects_duplicates_and_skips_failed(ctx):
    say("test_batch_rejects_duplicates_and_skips_failed")
    from paper_2103_09642_amd import edupic
    c, st = _mix()[1]
    g = _make(ctx, c, st, 0)
    with pytest.raises(edupic.EdpError) as ei:
        ctx.advance_steps([g, g], [1, 1])
    assert ei.value.code == edupic.EDP_EINVAL
    g.destroy()


def _descents(x, dx):
    """Fraction of neighbours in slot order whose cell index decreases."""
    c = np.floor(x / dx)
    return float(np.mean(c[1:] < c[:-1])) if c.size > 1 else 0.0


@pytest.mark.parametrize("mode", [0, 1], ids=["plain", "graph"])
def test_batched_sort_runs_only_for_cases_due(ctx, mode):
    """One batched step with the sort every 2 steps (ions every 2 N_SUB = 4):
    the case at step 0 is due for both species and comes out in cell order
    (up to one step of drift), the case at step 1 is not due and keeps its
    random slot order (about half the neighbours out of order)."""
    say(f"test_batched_sort_runs_only_for_cases_due mode={mode}")
    from paper_2103_09642_amd import edupic
    ctx.set_option(edupic.OPT_MODE, mode)
    ctx.set_option(edupic.OPT_SORT_EVERY, 2)
    try:
        c = base_case(n_init_e=0, n_init_i=0, weight=1e5, flags=["allow_unstable"], cap_e=80_000, cap_i=80_000,
                      n_grid=400, ion_subcycle=2, pressure_pa=10.0)
        st = random_state(20_000, 20_000, c["gap_m"], seed=77, te_ev=2.0, edge_cases=False)
        dx = c["gap_m"] / (c["n_grid"] - 1)
        for sp, key in ((0, "e"), (1, "i")):
            assert _descents(st[key]["x"], dx) > 0.4  # random order to begin with
        a, b = _make(ctx, c, st, 0), _make(ctx, c, st, 1)
        ctx.advance_steps([a, b], [1, 1])
        for sp in (0, 1):
            da, db = _descents(a.get_state(sp)["x"], dx), _descents(b.get_state(sp)["x"], dx)
            say(f"species {sp}: descents due {da:.4f}, not due {db:.4f}")
            # one step of drift after the sort: about 13% of electron and
            # 0.02% of ion neighbours out of order (a CPU model of this state)
            assert da < (0.25 if sp == 0 else 0.01), f"species {sp} of the case due was not sorted ({da})"
            assert db > 0.4, f"species {sp} of the case not due was sorted ({db})"
        a.destroy()
        b.destroy()
    finally:
        ctx.set_option(edupic.OPT_MODE, 0)
        ctx.set_option(edupic.OPT_SORT_EVERY, 100)
