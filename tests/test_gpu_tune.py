"""The sort-interval autotuner on library cases: it advances the real cases
under each candidate interval, so the state it leaves must be the state of
the same number of steps at any fixed interval, bit for bit (the step does
not depend on the sort interval)."""
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
        k, trials = tune.tune_sort_interval(ctx, gs, candidates=(5, 10, 40))
        assert k in (5, 10, 40) and len(trials) == 3 and all(t.rate > 0 for t in trials)
        assert tune.last_choice(ctx) == k
        # two half-length trials per candidate, each after its warm-up window
        total = sum(t.steps for t in trials) + 2 * sum(min(b, tune.MAX_TRIAL_STEPS)
                                                       for b in tune.trial_steps(gs, (5, 10, 40))[1].values())
        say(f"chosen {k}; rates {[round(t.rate / 1e9, 2) for t in trials]} G/s; {total} steps")
        tuned = [_result(g) for g in gs]
        assert all(r[3]["step"] == total for r in tuned)
        ctx.set_option(edupic.OPT_SORT_EVERY, 7)
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

