"""Autotuner for the batch runtime's schedule: the compaction + cell-sort
interval, the particle workgroups per CU and, for a batch of several cases,
the number of lockstep groups it runs as (and, when asked, the launch
mode: graph windows or plain launches).

* The sort every K steps trades its own cost (one pass over every particle
  array of the cases due) against the particle kernel's locality: between
  sorts, newborns are appended unsorted and particles drift between cells, so
  the streaming kernel slows down as the last sort recedes.
* The particle launches take, per case, a share of the chip's resident
  workgroup slots.  All of them hide the most memory latency, fewer leave
  each workgroup more chunks (each workgroup solves the field once per step)
  and the memory system less contention; which wins depends on the batch.

The best values depend on the workload -- a single case of 2e6 particles
per species is fastest near a 50-step interval, the 64-case batched set near
100-200; the dual-frequency set gains 7% from 4 workgroups per CU where the
batched set loses 2% -- and nothing in the results depends on any of them (a
step is bit-identical across sort intervals and launch shapes).  So the
tuner advances the real cases under each candidate in turn, losing no step,
times each trial with the device's own particle-step counters, and keeps the
fastest.  The knobs interact (4 workgroups per CU win at one sort interval
and lose at another), so when the calibration run says that every
combination fits in JOINT_BUDGET_SECONDS the tuner tries them all;
otherwise one knob at a time: the sort interval, then the workgroups per
CU at that interval.  Last, for a batch of several cases, the lockstep
groups (each on a stream of its own, one group's launch ramp and tail
overlapping another's streaming) at the chosen schedule.  The cases evolve while they are measured
(a seeded plasma loses or gains particles for many cycles), so the
candidates of a knob run in a mirrored order (A B C D D C B A) and each
one's rate pools its two trials: a linear drift of the throughput cancels.
Every trial is a whole number of every candidate's graph window, stretched
by a first calibration run to at least MIN_TRIAL_SECONDS, and among the
candidates within MARGIN of the fastest the one nearest the library's
default wins (so noise-level differences do not move a knob).
With `restore`, the tuner instead snapshots the cases' state once and
restores it before every trial and at the end: every trial then starts from
the same state, so the ranking reflects that state's regime (a joint search
runs dozens of RF cycles, over which a discharge can change enough to change
the ranking), and the cases come back unchanged.  A choice can be cached in
a JSON
file keyed by the batch's shape (case count, particle count bucket, grid
size, ion subcycling).

Host logic over the C ABI; `measure` can be replaced (tests use a model).
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass, replace
from typing import Callable, Dict, List, Optional, Sequence, Tuple

DEFAULT_CANDIDATES = (25, 50, 100, 200)  # sort intervals (steps)
DEFAULT_WG_CANDIDATES = (0, 4, 3)        # particle workgroups per CU (0: all that fit)
DEFAULT_GROUP_CANDIDATES = (2, 3, 4)     # lockstep groups of a multi-case batch
MAX_TRIAL_STEPS = 8000
MAX_TRIAL_STRETCH = 8       # at most this many windows per trial
MIN_TRIAL_SECONDS = 0.3     # calibration target per trial
MARGIN = 0.002              # rates this close to the fastest count as a tie
DEFAULTS = {"sort_every": 100, "part_wg_per_cu": 0, "groups": 2}
JOINT_BUDGET_SECONDS = 60.0  # all combinations tried together below this estimate
_chosen: Dict[int, Dict[str, int]] = {}  # last choice the tuner set, per context object


@dataclass
class Trial:
    interval: int        # the sort interval of the trial
    steps: int
    seconds: float
    particle_steps: int
    wg_per_cu: int = 0   # the particle workgroups per CU of the trial
    groups: int = 2      # the lockstep groups the trial ran as (set by the tuner)
    mode: int = -1       # the launch mode of the trial (1 graph, 0 plain; -1 as the context had it)

    @property
    def rate(self) -> float:
        return self.particle_steps / self.seconds if self.seconds > 0 else 0.0


def last_choice(ctx) -> Optional[int]:
    """The sort interval the tuner last set on this context (None if never)."""
    c = _chosen.get(id(ctx))
    return c["sort_every"] if c else None


def last_schedule(ctx) -> Optional[Dict[str, int]]:
    """Everything the tuner last set on this context (None if never)."""
    return _chosen.get(id(ctx))


def batch_key(cases: Sequence) -> str:
    """Shape of a batch: case count, total particles per species (power-of-two
    bucket), largest grid and the set of ion subcycles."""
    n = sum(max(1, c.counts()["n_e"]) for c in cases)
    ng = max(c.case["n_grid"] for c in cases)
    subs = sorted({int(c.case["ion_subcycle"]) for c in cases})
    return f"cases={len(cases)}:n_e~2^{int(round(math.log2(n)))}:ng={ng}:nsub={','.join(map(str, subs))}"


def trial_steps(cases: Sequence, candidates: Sequence[int]) -> Tuple[int, Dict[int, int]]:
    """A common timed length for every sort-interval candidate: a whole number
    of each candidate's graph window (interval x N_SUB of every case), capped;
    and each candidate's window."""
    subs = {int(c.case["ion_subcycle"]) for c in cases}
    base = {}
    for k in candidates:
        b = 1
        for s in subs:
            b = math.lcm(b, k * s)
        base[k] = b
    common = 1
    for b in base.values():
        common = math.lcm(common, b)
    steps = common if common <= MAX_TRIAL_STEPS else max(base.values())
    steps = min(max(steps, max(base.values())), MAX_TRIAL_STEPS)
    return steps, base


def measure(ctx, cases: Sequence, interval: int, steps: int, warm_steps: int, wg_per_cu: int = 0) -> Trial:
    """Advance `cases` by warm_steps (graph capture, first sort) and then by
    `steps` timed steps with the given schedule."""
    from . import edupic
    ctx.set_option(edupic.OPT_SORT_EVERY, interval)
    ctx.set_option(edupic.OPT_PART_WG_PER_CU, wg_per_cu)
    if warm_steps > 0:
        ctx.advance_steps(list(cases), [warm_steps] * len(cases))
    ctx.sync()
    c0 = [c.counts() for c in cases]
    t0 = time.perf_counter()
    ctx.advance_steps(list(cases), [steps] * len(cases))
    ctx.sync()
    t1 = time.perf_counter()
    c1 = [c.counts() for c in cases]
    ps = sum((b["psteps_e"] - a["psteps_e"]) + (b["psteps_i"] - a["psteps_i"]) for a, b in zip(c0, c1))
    return Trial(interval, steps, t1 - t0, ps, wg_per_cu)


def _mirrored(values: Sequence[int], trial: Callable[[int], Trial]) -> List[Trial]:
    """Trials of every value in the order A B .. B A, pooled per value."""
    runs = [(v, trial(v)) for v in list(values) + list(reversed(values))]
    out = []
    for v in values:
        mine = [t for w, t in runs if w == v]
        out.append(replace(mine[0], steps=sum(t.steps for t in mine), seconds=sum(t.seconds for t in mine),
                           particle_steps=sum(t.particle_steps for t in mine)))
    return out


def _pick(trials: List[Trial], attr: str, default: int, distance: Callable[[int], float]) -> int:
    """Among the trials within MARGIN of the fastest, the value nearest the
    library default (the default itself when it is among them): a tie in
    the evidence keeps the schedule closest to the default."""
    top = max(t.rate for t in trials)
    near = [getattr(t, attr) for t in trials if t.rate >= top / (1.0 + MARGIN)]
    return min(near, key=lambda v: (distance(v), v))


def _dist_sort(k):
    return abs(math.log(k / DEFAULTS["sort_every"]))


def _dist_wg(w):
    return 0.0 if w == 0 else 1.0 / w


def _dist_groups(g):
    return abs(g - DEFAULTS["groups"])


def _check(candidates, lo, what):
    if not candidates or any(int(k) < lo for k in candidates):
        raise ValueError(f"{what} candidates must be >= {lo}")


def _apply(ctx, sort_every: int, wg: int, groups: int, mode: Optional[int] = None):
    from . import edupic
    ctx.set_option(edupic.OPT_SORT_EVERY, sort_every)
    ctx.set_option(edupic.OPT_PART_WG_PER_CU, wg)
    ctx.set_option(edupic.OPT_GROUPS, groups)
    _chosen[id(ctx)] = {"sort_every": sort_every, "part_wg_per_cu": wg, "groups": groups}
    if mode is not None:
        ctx.set_option(edupic.OPT_MODE, mode)
        _chosen[id(ctx)]["mode"] = mode


def snapshot(cases: Sequence) -> List:
    """Each case's particles of both species and its step (host copies)."""
    return [(c.get_state(0), c.get_state(1), c.counts()["step"]) for c in cases]


def restore(cases: Sequence, snap: List):
    for c, (e, i, step) in zip(cases, snap):
        c.set_state(0, e, step)
        c.set_state(1, i, step)


def tune_schedule(ctx, cases: Sequence, candidates: Sequence[int] = DEFAULT_CANDIDATES,
                  wg_candidates: Sequence[int] = DEFAULT_WG_CANDIDATES, cache_path: Optional[str] = None,
                  measure_fn: Optional[Callable[..., Trial]] = None,
                  restore_state: bool = False,
                  group_candidates: Sequence[int] = DEFAULT_GROUP_CANDIDATES,
                  mode_candidates: Sequence[int] = ()) -> Tuple[Dict[str, int], List[Trial]]:
    """Pick the fastest sort interval, then the fastest particle workgroups
    per CU at that interval, then (a batch of several cases) the fastest
    lockstep groups, and set them on the context.  Returns ({"sort_every",
    "part_wg_per_cu", "groups"}, trials); no trials when the cache answered.
    Empty `wg_candidates` leave the workgroups at all that fit, empty
    `group_candidates` (or a batch with fewer cases than two of them) the
    groups at 2.  Every trial
    before the groups stage runs with 2 groups.  With `mode_candidates`
    (launch modes: 1 graph windows, 0 plain launches) the last stage tries
    every group count in every mode -- several groups' graphs can overlap
    worse than their plain launches -- and the choice gains a "mode".  With
    restore_state every trial starts from the cases' state at the call, and
    the cases end in it."""
    from . import edupic
    _check(candidates, 1, "sort interval")
    if wg_candidates:
        _check(wg_candidates, 0, "workgroup")
    if group_candidates and any(int(g) not in (1, 2, 3, 4) for g in group_candidates):
        raise ValueError("group candidates must be 1..4")
    if any(int(m) not in (0, 1) for m in mode_candidates):
        raise ValueError("mode candidates must be 0 or 1")
    # more groups than cases run as one group per case: those candidates are
    # the same as the case count
    gs = sorted({min(int(g), len(cases)) for g in group_candidates})
    gs = gs if len(gs) > 1 else []
    ms = [int(m) for m in mode_candidates]
    key = batch_key(cases) + (":wg" if wg_candidates else "") + (":groups" if gs else "") + (":mode" if ms else "")
    cache: Dict[str, Dict] = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            hit = cache[key]
            _apply(ctx, int(hit["sort_every"]), int(hit.get("part_wg_per_cu", 0)),
                   int(hit.get("groups", DEFAULTS["groups"])), hit.get("mode"))
            return dict(_chosen[id(ctx)]), []
    ctx.set_option(edupic.OPT_GROUPS, DEFAULTS["groups"])
    steps, base = trial_steps(cases, candidates)
    measure_one = measure_fn or measure
    snap = snapshot(cases) if restore_state else None

    def run(*a):
        if snap is not None:
            restore(cases, snap)
        return measure_one(*a)
    # calibration (not counted; also a warm-up): stretch the trials of a fast
    # batch to MIN_TRIAL_SECONDS, by whole windows
    k0 = int(candidates[0])
    cal = run(ctx, cases, k0, steps, min(base[k0], MAX_TRIAL_STEPS), 0)
    if 0 < cal.seconds < MIN_TRIAL_SECONDS:
        steps *= min(MAX_TRIAL_STRETCH, math.ceil(MIN_TRIAL_SECONDS / cal.seconds))
    per_trial = cal.seconds * steps / cal.steps if cal.steps else 0.0
    ks = [int(k) for k in candidates]
    ws = [int(w) for w in wg_candidates] or [0]
    combos = [(k, w) for k in ks for w in ws]
    if len(combos) > 1 and 2 * len(combos) * per_trial <= JOINT_BUDGET_SECONDS:
        # every combination, in one mirrored sequence; ties go to the
        # combination nearest the defaults
        idx = list(range(len(combos)))
        trials = _mirrored(idx, lambda i: run(ctx, cases, combos[i][0], steps, min(base[combos[i][0]], MAX_TRIAL_STEPS),
                                              combos[i][1]))
        top = max(t.rate for t in trials)
        near = [t for t in trials if t.rate >= top / (1.0 + MARGIN)]
        win = min(near, key=lambda t: (_dist_sort(t.interval) + _dist_wg(t.wg_per_cu), t.interval, t.wg_per_cu))
        best_k, best_w = win.interval, win.wg_per_cu
    else:
        trials = _mirrored(ks, lambda k: run(ctx, cases, k, steps, min(base[k], MAX_TRIAL_STEPS), 0))
        best_k = _pick(trials, "interval", DEFAULTS["sort_every"], _dist_sort)
        warm = min(base[best_k], MAX_TRIAL_STEPS)
        best_w = 0
        if wg_candidates:
            wt = _mirrored(ws, lambda w: run(ctx, cases, best_k, steps, warm, w))
            best_w = _pick(wt, "wg_per_cu", DEFAULTS["part_wg_per_cu"], _dist_wg)
            trials += wt
    # the groups these trials ran as (a batch smaller than the option runs
    # as one group per case)
    trials = [replace(t, groups=min(DEFAULTS["groups"], len(cases))) for t in trials]
    best_g = DEFAULTS["groups"]
    best_m = None
    if ms:
        # every group count (the default alone for a single case) in every mode
        combos = [(g, m) for g in (gs or [best_g]) for m in ms]

        def gm_trial(i):
            g, m = combos[i]
            ctx.set_option(edupic.OPT_GROUPS, g)
            ctx.set_option(edupic.OPT_MODE, m)
            t = run(ctx, cases, best_k, steps, min(base[best_k], MAX_TRIAL_STEPS), best_w)
            return replace(t, groups=min(g, len(cases)), mode=m)
        gt = _mirrored(list(range(len(combos))), gm_trial)
        top = max(t.rate for t in gt)
        near = [i for i, t in enumerate(gt) if t.rate >= top / (1.0 + MARGIN)]
        # a tie goes to the default groups, then to graph windows
        best_g, best_m = combos[min(near, key=lambda i: (_dist_groups(combos[i][0]), -combos[i][1]))]
        trials += gt
    elif gs:
        def group_trial(g):
            ctx.set_option(edupic.OPT_GROUPS, g)
            return replace(run(ctx, cases, best_k, steps, min(base[best_k], MAX_TRIAL_STEPS), best_w), groups=g)
        gt = _mirrored(gs, group_trial)
        best_g = _pick(gt, "groups", DEFAULTS["groups"], _dist_groups)
        trials += gt
    if snap is not None:
        restore(cases, snap)
    _apply(ctx, best_k, best_w, best_g, best_m)
    if cache_path:
        cache[key] = {"sort_every": best_k, "part_wg_per_cu": best_w, "groups": best_g,
                      "trials": [dict(asdict(t), rate=t.rate) for t in trials]}
        if best_m is not None:
            cache[key]["mode"] = best_m
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return dict(_chosen[id(ctx)]), trials


def tune_sort_interval(ctx, cases: Sequence, candidates: Sequence[int] = DEFAULT_CANDIDATES,
                       cache_path: Optional[str] = None,
                       measure_fn: Optional[Callable[..., Trial]] = None) -> Tuple[int, List[Trial]]:
    """The sort interval alone (all workgroups that fit, 2 groups)."""
    choice, trials = tune_schedule(ctx, cases, candidates, (), cache_path, measure_fn, group_candidates=())
    return choice["sort_every"], trials
