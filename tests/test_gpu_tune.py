"""The schedule autotuner on library cases: it advances the real cases under
each candidate sort interval and workgroup count, so the state it leaves
must be the state of the same number of steps under any fixed schedule,
bit for bit (a step depends neither on the sort interval nor on the launch
shape)."""
import pytest

from gpu_common import gpu_context, say
from paper_2103_09642_amd import tune
from test_gpu_batch import _make, _mix, _result, _same

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(xs_default):
    c = gpu_context()
    c.set_xsec(xs_default)
    return c


def test_tuning_loses_no_step_and_changes_nothing(ctx):
    say("test_tuning_loses_no_step_and_changes_nothing")
    from paper_2103_09642_amd import edupic
    mix = _mix()[:2]  # N_SUB 20 and 5
    ctx.set_option(edupic.OPT_MODE, 1)
    try:
        gs = [_make(ctx, c, st, 0) for c, st in mix]
        choice, trials = tune.tune_schedule(ctx, gs, candidates=(5, 10, 40), wg_candidates=(0, 2))
        assert choice["sort_every"] in (5, 10, 40) and choice["part_wg_per_cu"] in (0, 2)
        assert tune.last_schedule(ctx) == choice
        # one knob at a time (3 + 2) or, for cases this cheap, every
        # combination (3 x 2), then the groups (2 and 3 for these two cases:
        # capped at 2, nothing to try)
        assert len(trials) in (5, 6) and all(t.rate > 0 for t in trials)
        say(f"chosen {choice}; rates {[round(t.rate / 1e9, 2) for t in trials]} G/s")
        tuned = [_result(g) for g in gs]
        total = tuned[0][3]["step"]
        assert total > 0 and all(r[3]["step"] == total for r in tuned)
        ctx.set_option(edupic.OPT_SORT_EVERY, 7)
        ctx.set_option(edupic.OPT_PART_WG_PER_CU, 1)
        for (c, st), r in zip(mix, tuned):
            g = _make(ctx, c, st, 0)
            g.advance_steps(total)
            _same(_result(g), r, f"n_grid={c['n_grid']}")
            g.destroy()
        for g in gs:
            g.destroy()
    finally:
        ctx.set_option(edupic.OPT_MODE, 0)
        ctx.set_option(edupic.OPT_SORT_EVERY, 100)
        ctx.set_option(edupic.OPT_PART_WG_PER_CU, 0)


def test_tuning_with_restore_leaves_the_cases_unchanged(ctx):
    """restore_state: every trial starts from the cases' state at the call,
    and the cases come back to it, bit for bit, at the same step."""
    say("test_tuning_with_restore_leaves_the_cases_unchanged")
    from paper_2103_09642_amd import edupic
    mix = _mix()[:2]
    ctx.set_option(edupic.OPT_MODE, 1)
    try:
        gs = [_make(ctx, c, st, 3) for c, st in mix]
        for g in gs:
            g.advance_steps(40)
        before = [_result(g) for g in gs]
        choice, trials = tune.tune_schedule(ctx, gs, candidates=(5, 10), wg_candidates=(0, 2), restore_state=True)
        assert len(trials) == 4 and all(t.rate > 0 for t in trials)
        for g, b in zip(gs, before):
            a = _result(g)
            assert a[3]["step"] == b[3]["step"] == 43
            for sp in (0, 1):
                for k in ("uid", "x", "vx", "vy", "vz"):
                    assert (a[sp][k] == b[sp][k]).all(), (sp, k)
            g.destroy()
    finally:
        ctx.set_option(edupic.OPT_MODE, 0)
        ctx.set_option(edupic.OPT_SORT_EVERY, 100)
        ctx.set_option(edupic.OPT_PART_WG_PER_CU, 0)


def test_group_stage_on_library_cases(ctx):
    """The lockstep-groups stage on three library cases: 1, 2 and 3 groups
    are tried in a mirrored order at the chosen schedule, the choice is set
    on the context, and with restore_state the cases come back unchanged."""
    say("test_group_stage_on_library_cases")
    from paper_2103_09642_amd import edupic
    mix = _mix()[:3]
    ctx.set_option(edupic.OPT_MODE, 1)
    try:
        gs = [_make(ctx, c, st, 0) for c, st in mix]
        before = [_result(g) for g in gs]
        choice, trials = tune.tune_schedule(ctx, gs, candidates=(10,), wg_candidates=(),
                                            group_candidates=(1, 2, 3, 4), restore_state=True)
        assert [t.groups for t in trials] == [2, 1, 2, 3] and all(t.rate > 0 for t in trials)
        assert choice["groups"] in (1, 2, 3) and tune.last_schedule(ctx) == choice
        say(f"chosen {choice}; rates {[round(t.rate / 1e9, 2) for t in trials]} G/s")
        for g, b in zip(gs, before):
            a = _result(g)
            assert a[3]["step"] == b[3]["step"] == 0
            for sp in (0, 1):
                for k in ("uid", "x", "vx", "vy", "vz"):
                    assert (a[sp][k] == b[sp][k]).all(), (sp, k)
            g.destroy()
    finally:
        ctx.set_option(edupic.OPT_MODE, 0)
        ctx.set_option(edupic.OPT_SORT_EVERY, 100)
        ctx.set_option(edupic.OPT_GROUPS, 2)


def test_workgroup_option_is_validated(ctx):
    from paper_2103_09642_amd import edupic
    say("test_workgroup_option_is_validated")
    for bad in (-1, 65):
        with pytest.raises(edupic.EdpError):
            ctx.set_option(edupic.OPT_PART_WG_PER_CU, bad)
    with pytest.raises(edupic.EdpError):
        ctx.set_option(10, 64)  # no such option
