"""The sort-interval autotuner's host logic on model batches (no GPU): the
trial lengths, the choice of the fastest candidate, and its JSON cache."""
import json

import pytest

from paper_2103_09642_amd import edupic, tune


class FakeCtx:
    def __init__(self):
        self.options = {}

    def set_option(self, key, value):
        self.options[key] = value


class FakeCase:
    def __init__(self, n_e, n_grid, nsub):
        self.case = {"n_grid": n_grid, "ion_subcycle": nsub}
        self._n = n_e

    def counts(self):
        return {"n_e": self._n}


def model(cost):
    """A measure function from a per-step cost model: seconds = steps x cost(k)."""
    calls = []

    def run(ctx, cases, k, steps, warm, wg=0):
        calls.append((k, steps, warm))
        return tune.Trial(k, steps, steps * cost(k), steps * 1000, wg)
    return run, calls


def test_trial_lengths_cover_whole_graph_windows():
    cases = [FakeCase(2_000_000, 1000, 20)]
    steps, base = tune.trial_steps(cases, (25, 50, 100, 200))
    assert base == {25: 500, 50: 1000, 100: 2000, 200: 4000}
    assert steps == 4000 and all(steps % b == 0 for b in base.values())
    # subcycles whose windows do not share a short multiple: capped
    steps, base = tune.trial_steps([FakeCase(1000, 400, 7), FakeCase(1000, 400, 11)], (25, 50, 100, 200))
    assert base[200] == 200 * 77 and steps == tune.MAX_TRIAL_STEPS


def test_picks_the_fastest_and_sets_it():
    ctx = FakeCtx()
    # sort cost 70/k per step plus a locality loss growing with k: best at 50
    run, calls = model(lambda k: 22.0 + 70.0 / k + 0.03 * k)
    k, trials = tune.tune_sort_interval(ctx, [FakeCase(2_000_000, 1000, 20)], measure_fn=run)
    assert k == 50 and ctx.options[edupic.OPT_SORT_EVERY] == 50
    assert [t.interval for t in trials] == [25, 50, 100, 200]
    # a calibration run, then the mirrored order with whole-window trials
    # pooled per candidate
    assert [k for k, _, _ in calls] == [25] + [25, 50, 100, 200, 200, 100, 50, 25]
    assert all(st == 4000 for _, st, _ in calls) and all(t.steps == 8000 for t in trials)
    assert [w for _, _, w in calls[1:5]] == [500, 1000, 2000, 4000]


def test_mirrored_order_cancels_a_linear_drift():
    """The throughput falls 5% per trial while the cases evolve, and the
    intervals themselves make no difference: pooled rates come out equal, so
    the drift does not pick the interval measured first."""
    ctx = FakeCtx()
    n = [0]

    def run(ctx_, cases, k, steps, warm, wg=0):
        t = tune.Trial(k, steps, steps * 1.0, int(steps * 1000 * (1.0 - 0.05 * n[0])), wg)
        n[0] += 1
        return t
    k, trials = tune.tune_sort_interval(ctx, [FakeCase(1_000_000, 1000, 20)], measure_fn=run)
    rates = [t.rate for t in trials]
    assert max(rates) - min(rates) < 1e-5 * max(rates)  # (integer particle-step counts)


def test_cache_answers_the_same_batch_shape(tmp_path):
    path = str(tmp_path / "tune.json")
    ctx = FakeCtx()
    run, calls = model(lambda k: 1.0 + abs(k - 100) * 1e-3)
    k, trials = tune.tune_sort_interval(ctx, [FakeCase(300_000, 800, 20)] * 3, cache_path=path, measure_fn=run)
    assert k == 100 and len(trials) == 4 and len(calls) == 9
    saved = json.load(open(path))
    (key, entry), = saved.items()
    assert entry["sort_every"] == 100 and "cases=3" in key
    ctx2 = FakeCtx()
    run2, calls2 = model(lambda k: 1.0)
    k2, trials2 = tune.tune_sort_interval(ctx2, [FakeCase(300_000, 800, 20)] * 3, cache_path=path, measure_fn=run2)
    assert k2 == 100 and trials2 == [] and calls2 == [] and ctx2.options[edupic.OPT_SORT_EVERY] == 100
    # another shape is tuned afresh and added
    tune.tune_sort_interval(FakeCtx(), [FakeCase(300_000, 800, 20)], cache_path=path, measure_fn=run2)
    assert len(json.load(open(path))) == 2


def test_schedule_tunes_the_workgroups_at_the_chosen_interval(tmp_path):
    """Second knob: with the interval fixed at the winner, the workgroups
    per CU (0: all that fit) are tried in a mirrored order as well."""
    calls = []

    def run(ctx, cases, k, steps, warm, wg=0):
        calls.append((k, wg, warm))
        cost = 22.0 + 70.0 / k + 0.03 * k + {0: 1.0, 4: 0.0, 3: 0.5}[wg]
        return tune.Trial(k, steps, steps * cost, steps * 1000, wg)
    ctx = FakeCtx()
    path = str(tmp_path / "t.json")
    # a slow batch (above the joint budget): one knob at a time
    tune.JOINT_BUDGET_SECONDS, saved = 0.0, tune.JOINT_BUDGET_SECONDS
    try:
        choice, trials = tune.tune_schedule(ctx, [FakeCase(1_000_000, 1000, 20)] * 4, cache_path=path,
                                            measure_fn=run, group_candidates=())
    finally:
        tune.JOINT_BUDGET_SECONDS = saved
    assert choice == {"sort_every": 50, "part_wg_per_cu": 4, "groups": 2}
    assert ctx.options[edupic.OPT_SORT_EVERY] == 50 and ctx.options[edupic.OPT_PART_WG_PER_CU] == 4
    assert [(k, w) for k, w, _ in calls[9:15]] == [(50, 0), (50, 4), (50, 3), (50, 3), (50, 4), (50, 0)]
    assert all(warm == 1000 for _, _, warm in calls[9:])
    assert len(trials) == 7
    entry, = json.load(open(path)).values()
    assert entry["sort_every"] == 50 and entry["part_wg_per_cu"] == 4
    ctx2 = FakeCtx()
    assert tune.tune_schedule(ctx2, [FakeCase(1_000_000, 1000, 20)] * 4, cache_path=path, measure_fn=run,
                              group_candidates=())[1] == []
    assert ctx2.options[edupic.OPT_PART_WG_PER_CU] == 4


def test_short_trials_are_stretched_by_whole_windows():
    """A fast batch: the calibration run takes 1/10 of MIN_TRIAL_SECONDS, so
    every trial runs 10 windows of the common length (capped)."""
    steps_seen = []

    def run(ctx, cases, k, steps, warm, wg=0):
        steps_seen.append(steps)
        return tune.Trial(k, steps, steps * tune.MIN_TRIAL_SECONDS / 40000, steps * 1000, wg)
    tune.tune_sort_interval(FakeCtx(), [FakeCase(10_000, 200, 20)], measure_fn=run)
    assert steps_seen[0] == 4000
    assert all(st == 4000 * min(10, tune.MAX_TRIAL_STRETCH) for st in steps_seen[1:])


def test_a_default_within_the_margin_is_kept():
    """Noise-level differences do not move a knob off the library default."""
    def run(ctx, cases, k, steps, warm, wg=0):
        gain = 1.0 + (0.001 if wg == 4 else 0.0) + (0.02 if wg == 3 else 0.0)
        return tune.Trial(k, steps, steps / gain, steps * 1000, wg)
    choice, _ = tune.tune_schedule(FakeCtx(), [FakeCase(2_000_000, 1000, 20)], measure_fn=run)
    assert choice == {"sort_every": 100, "part_wg_per_cu": 3, "groups": 2}
    choice, _ = tune.tune_schedule(FakeCtx(), [FakeCase(2_000_000, 1000, 20)], wg_candidates=(0, 4),
                                   measure_fn=run)
    assert choice == {"sort_every": 100, "part_wg_per_cu": 0, "groups": 2}


def test_a_tie_goes_to_the_value_nearest_the_default():
    """Intervals 25 and 50 within the margin, both well ahead of 100: 50
    (nearer 100) is kept."""
    def run(ctx, cases, k, steps, warm, wg=0):
        gain = {25: 1.0301, 50: 1.03, 100: 1.0, 200: 0.95}[k]
        return tune.Trial(k, steps, steps / gain, steps * 1000, wg)
    k, _ = tune.tune_sort_interval(FakeCtx(), [FakeCase(2_000_000, 1000, 20)], measure_fn=run)
    assert k == 50


def test_cheap_batches_search_every_combination():
    """4 workgroups per CU win only at a 25-step interval: one knob at a time
    would keep (50, all); trials this short fit the joint budget, so every
    combination is tried and (25, 4) found."""
    seen = []

    def rate(k, w):
        r = {25: 1.0, 50: 1.05, 100: 1.02, 200: 0.97}[k]
        if w == 4:
            r *= 1.08 if k == 25 else 0.99
        return r

    def run(ctx, cases, k, steps, warm, wg=0):
        seen.append((k, wg))
        return tune.Trial(k, steps, steps * 1e-6 / rate(k, wg), steps, wg)
    choice, trials = tune.tune_schedule(FakeCtx(), [FakeCase(2_000_000, 1000, 20)], measure_fn=run)
    assert choice == {"sort_every": 25, "part_wg_per_cu": 4, "groups": 2}
    assert len(trials) == 4 * 3 and len(seen) == 1 + 2 * 12


def test_rejects_bad_candidates():
    with pytest.raises(ValueError):
        tune.tune_sort_interval(FakeCtx(), [FakeCase(1000, 100, 5)], candidates=(0, 10))
    with pytest.raises(ValueError):
        tune.tune_schedule(FakeCtx(), [FakeCase(1000, 100, 5)], wg_candidates=(4, -1))


def test_groups_are_tuned_last_for_a_batch_of_cases(tmp_path):
    """Last stage, only for several cases: the lockstep groups at the chosen
    schedule, in a mirrored order, capped at the case count; every earlier
    trial runs with 2 groups; the choice is set and cached."""
    calls = []

    def run(ctx, cases, k, steps, warm, wg=0):
        g = ctx.options[edupic.OPT_GROUPS]
        calls.append((k, wg, g))
        cost = 22.0 + 70.0 / k + 0.03 * k + {2: 1.0, 3: 0.0, 4: 0.4}[g]
        return tune.Trial(k, steps, steps * cost, steps * 1000, wg)
    ctx = FakeCtx()
    path = str(tmp_path / "g.json")
    cases = [FakeCase(300_000, 1000, 20)] * 5
    choice, trials = tune.tune_schedule(ctx, cases, wg_candidates=(), cache_path=path, measure_fn=run)
    assert choice == {"sort_every": 50, "part_wg_per_cu": 0, "groups": 3}
    assert ctx.options[edupic.OPT_GROUPS] == 3
    assert all(g == 2 for _, _, g in calls[:9])
    assert [g for _, _, g in calls[9:]] == [2, 3, 4, 4, 3, 2]
    assert all(k == 50 for k, _, _ in calls[9:])
    assert [t.groups for t in trials] == [2] * 4 + [2, 3, 4]
    assert json.load(open(path))[tune.batch_key(cases) + ":groups"]["groups"] == 3
    # two cases: 3 and 4 groups are 2 groups, nothing to try
    calls.clear()
    choice, trials = tune.tune_schedule(FakeCtx(), cases[:2], wg_candidates=(), measure_fn=run)
    assert choice["groups"] == 2 and len(trials) == 4 and all(g == 2 for _, _, g in calls)
    # one case runs alone whatever the option says
    _, trials = tune.tune_schedule(FakeCtx(), cases[:1], wg_candidates=(), measure_fn=run)
    assert [t.groups for t in trials] == [1] * 4
    with pytest.raises(ValueError):
        tune.tune_schedule(FakeCtx(), cases, group_candidates=(2, 5), measure_fn=run)


def test_modes_are_tuned_with_the_groups():
    """With mode candidates the last stage tries every group count in both
    launch modes (graph windows and plain launches) and sets the fastest
    pair; a tie goes to the default groups and then to graph windows."""
    calls = []

    def run(ctx, cases, k, steps, warm, wg=0):
        g, m = ctx.options[edupic.OPT_GROUPS], ctx.options.get(edupic.OPT_MODE, 1)
        calls.append((g, m))
        # plain launches overlap better at 4 groups, graphs win below
        rate = {(2, 1): 1.00, (2, 0): 0.99, (3, 1): 1.02, (3, 0): 1.01, (4, 1): 1.01, (4, 0): 1.06}[(g, m)]
        return tune.Trial(k, steps, steps * 1e-6 / rate, steps, wg)
    ctx = FakeCtx()
    cases = [FakeCase(300_000, 1000, 20)] * 6
    choice, trials = tune.tune_schedule(ctx, cases, candidates=(100,), wg_candidates=(), measure_fn=run,
                                        mode_candidates=(1, 0))
    assert choice == {"sort_every": 100, "part_wg_per_cu": 0, "groups": 4, "mode": 0}
    assert ctx.options[edupic.OPT_MODE] == 0 and ctx.options[edupic.OPT_GROUPS] == 4
    assert [(t.groups, t.mode) for t in trials[-6:]] == [(2, 1), (2, 0), (3, 1), (3, 0), (4, 1), (4, 0)]
    # a tie keeps the default groups in graph windows
    def flat(ctx, cases, k, steps, warm, wg=0):
        return tune.Trial(k, steps, steps * 1e-6, steps, wg)
    choice, _ = tune.tune_schedule(FakeCtx(), cases, candidates=(100,), wg_candidates=(), measure_fn=flat,
                                   mode_candidates=(1, 0))
    assert choice["groups"] == 2 and choice["mode"] == 1
    # a single case: the modes alone
    choice, trials = tune.tune_schedule(FakeCtx(), cases[:1], candidates=(100,), wg_candidates=(), measure_fn=flat,
                                        mode_candidates=(1, 0))
    assert "mode" in choice and [t.mode for t in trials[-2:]] == [1, 0]
    with pytest.raises(ValueError):
        tune.tune_schedule(FakeCtx(), cases, mode_candidates=(2,), measure_fn=flat)
