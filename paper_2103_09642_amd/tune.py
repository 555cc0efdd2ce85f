"""Autotuner for the batch runtime's schedule: the compaction + cell-sort
interval and the particle workgroups per CU.

* The sort every K steps trades its own cost (one pass over every particle
  array of the cases due) against the particle kernel's locality: between
  sorts, newborns are appended unsorted and particles drift between cells, so
  the streaming kernel slows down as the last sort recedes.
* The particle launches take, per case, a share of the chip's resident
  workgroup slots.  All of them (5 per CU for electrons) hide the most memory
  latency, fewer leave each workgroup more chunks and the memory system less
  contention; which wins depends on the batch.

The best values depend on the workload -- a single case of 2e6 particles
per species is fastest near a 50-step interval, the 64-case batched set near
100-200; the dual-frequency set gains 7% from 4 workgroups per CU where the
batched set loses 2% -- and nothing in the results depends on either (a step
is bit-identical across sort intervals and launch shapes).  So the tuner
advances the real cases under each candidate in turn, losing no step, times
each trial with the device's own particle-step counters, and keeps the
fastest: first the sort interval, then the workgroups per CU at that
interval.  The cases evolve while they are measured (a seeded plasma loses
or gains particles for many cycles), so the candidates of a knob run in a
mirrored order (A B C D D C B A) and each one's rate pools its two trials: a
linear drift of the throughput cancels.  A choice can be cached in a JSON
file keyed by the batch's shape (case count, particle count bucket, grid
size, ion subcycling).

Host logic over the C ABI; `measure` can be replaced (tests use a model).
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass
from typing import Callable, Dict, List, Optional, Sequence, Tuple

DEFAULT_CANDIDATES = (25, 50, 100, 200)  # sort intervals (steps)
DEFAULT_WG_CANDIDATES = (0, 4, 3)        # particle workgroups per CU (0: all that fit)
MAX_TRIAL_STEPS = 8000
_chosen: Dict[int, Dict[str, int]] = {}  # last choice the tuner set, per context object


@dataclass
class Trial:
    interval: int        # the sort interval of the trial
    steps: int
    seconds: float
    particle_steps: int
    wg_per_cu: int = 0   # the particle workgroups per CU of the trial

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
        out.append(Trial(mine[0].interval, sum(t.steps for t in mine), sum(t.seconds for t in mine),
                         sum(t.particle_steps for t in mine), mine[0].wg_per_cu))
    return out


def _check(candidates, lo, what):
    if not candidates or any(int(k) < lo for k in candidates):
        raise ValueError(f"{what} candidates must be >= {lo}")


def _apply(ctx, sort_every: int, wg: int):
    from . import edupic
    ctx.set_option(edupic.OPT_SORT_EVERY, sort_every)
    ctx.set_option(edupic.OPT_PART_WG_PER_CU, wg)
    _chosen[id(ctx)] = {"sort_every": sort_every, "part_wg_per_cu": wg}


def tune_schedule(ctx, cases: Sequence, candidates: Sequence[int] = DEFAULT_CANDIDATES,
                  wg_candidates: Sequence[int] = DEFAULT_WG_CANDIDATES, cache_path: Optional[str] = None,
                  measure_fn: Optional[Callable[..., Trial]] = None) -> Tuple[Dict[str, int], List[Trial]]:
    """Pick the fastest sort interval, then the fastest particle workgroups
    per CU at that interval, and set both on the context.  Returns
    ({"sort_every", "part_wg_per_cu"}, trials); no trials when the cache
    answered.  Empty `wg_candidates` leave the workgroups at all that fit."""
    _check(candidates, 1, "sort interval")
    if wg_candidates:
        _check(wg_candidates, 0, "workgroup")
    key = batch_key(cases) + (":wg" if wg_candidates else "")
    cache: Dict[str, Dict] = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            hit = cache[key]
            _apply(ctx, int(hit["sort_every"]), int(hit.get("part_wg_per_cu", 0)))
            return dict(_chosen[id(ctx)]), []
    steps, base = trial_steps(cases, candidates)
    half = max(1, steps // 2)
    run = measure_fn or measure
    trials = _mirrored([int(k) for k in candidates],
                       lambda k: run(ctx, cases, k, half, min(base[k], MAX_TRIAL_STEPS), 0))
    best_k = max(trials, key=lambda t: t.rate).interval
    best_w = 0
    if wg_candidates:
        wt = _mirrored([int(w) for w in wg_candidates],
                       lambda w: run(ctx, cases, best_k, half, min(base[best_k], MAX_TRIAL_STEPS), w))
        best_w = max(wt, key=lambda t: t.rate).wg_per_cu
        trials += wt
    _apply(ctx, best_k, best_w)
    if cache_path:
        cache[key] = {"sort_every": best_k, "part_wg_per_cu": best_w,
                      "trials": [dict(asdict(t), rate=t.rate) for t in trials]}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return dict(_chosen[id(ctx)]), trials


def tune_sort_interval(ctx, cases: Sequence, candidates: Sequence[int] = DEFAULT_CANDIDATES,
                       cache_path: Optional[str] = None,
                       measure_fn: Optional[Callable[..., Trial]] = None) -> Tuple[int, List[Trial]]:
    """The sort interval alone (the workgroups stay at all that fit)."""
    choice, trials = tune_schedule(ctx, cases, candidates, (), cache_path, measure_fn)
    return choice["sort_every"], trials
