"""Autotuner for the batch runtime's compaction + cell-sort interval.

The sort every K steps trades its own cost (one pass over every particle
array of the cases due) against the particle kernel's locality: between
sorts, newborns are appended unsorted and particles drift between cells, so
the streaming kernel slows down as the last sort recedes.  The best K
depends on the workload -- a single case of 2e6 particles per species is
fastest near 50 steps, the 64-case batched set near 100 -- and nothing in
the results depends on it (a step is bit-identical across sort intervals).
So the tuner advances the real cases under each candidate interval in turn,
losing no step, times each trial with the device's own particle-step
counters, and keeps the fastest.  The cases evolve while they are measured
(a seeded plasma loses or gains particles for many cycles), so the
candidates run in a mirrored order (A B C D D C B A) and each one's rate
pools its two trials: a linear drift of the throughput cancels.  A choice can be cached in a JSON file
keyed by the batch's shape (case count, particle count bucket, grid size,
ion subcycling).

Host logic over the C ABI; `measure` can be replaced (tests use a model).
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import asdict, dataclass
from typing import Callable, Dict, List, Optional, Sequence, Tuple

DEFAULT_CANDIDATES = (25, 50, 100, 200)
MAX_TRIAL_STEPS = 8000
_chosen: Dict[int, int] = {}  # last interval the tuner set, per context object


def last_choice(ctx) -> Optional[int]:
    """The interval the tuner last set on this context (None if never)."""
    return _chosen.get(id(ctx))


@dataclass
class Trial:
    interval: int
    steps: int
    seconds: float
    particle_steps: int

    @property
    def rate(self) -> float:
        return self.particle_steps / self.seconds if self.seconds > 0 else 0.0


def batch_key(cases: Sequence) -> str:
    """Shape of a batch: case count, total particles per species (power-of-two
    bucket), largest grid and the set of ion subcycles."""
    n = sum(max(1, c.counts()["n_e"]) for c in cases)
    ng = max(c.case["n_grid"] for c in cases)
    subs = sorted({int(c.case["ion_subcycle"]) for c in cases})
    return f"cases={len(cases)}:n_e~2^{int(round(math.log2(n)))}:ng={ng}:nsub={','.join(map(str, subs))}"


def trial_steps(cases: Sequence, candidates: Sequence[int]) -> Tuple[int, Dict[int, int]]:
    """A common timed length for every candidate: a whole number of each
    candidate's graph window (interval x N_SUB of every case), capped."""
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


def measure(ctx, cases: Sequence, interval: int, steps: int, warm_steps: int) -> Trial:
    """Advance `cases` by warm_steps (graph capture, first sort) and then by
    `steps` timed steps with the given interval."""
    from . import edupic
    ctx.set_option(edupic.OPT_SORT_EVERY, interval)
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
    return Trial(interval, steps, t1 - t0, ps)


def tune_sort_interval(ctx, cases: Sequence, candidates: Sequence[int] = DEFAULT_CANDIDATES,
                       cache_path: Optional[str] = None,
                       measure_fn: Optional[Callable[..., Trial]] = None) -> Tuple[int, List[Trial]]:
    """Pick the fastest sort interval for this batch and set it on the
    context.  Returns (interval, trials); no trials when the cache answered."""
    from . import edupic
    if not candidates or any(int(k) < 1 for k in candidates):
        raise ValueError("candidates must be positive step counts")
    key = batch_key(cases)
    cache: Dict[str, Dict] = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            k = int(cache[key]["sort_every"])
            ctx.set_option(edupic.OPT_SORT_EVERY, k)
            _chosen[id(ctx)] = k
            return k, []
    steps, base = trial_steps(cases, candidates)
    half = max(1, steps // 2)
    run = measure_fn or measure
    order = [int(k) for k in candidates] + [int(k) for k in reversed(candidates)]
    runs = [run(ctx, cases, k, half, min(base[k], MAX_TRIAL_STEPS)) for k in order]
    trials = []
    for k in candidates:
        mine = [t for t in runs if t.interval == int(k)]
        trials.append(Trial(int(k), sum(t.steps for t in mine), sum(t.seconds for t in mine),
                            sum(t.particle_steps for t in mine)))
    best = max(trials, key=lambda t: t.rate)
    ctx.set_option(edupic.OPT_SORT_EVERY, best.interval)
    _chosen[id(ctx)] = best.interval
    if cache_path:
        cache[key] = {"sort_every": best.interval, "trials": [dict(asdict(t), rate=t.rate) for t in trials]}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return best.interval, trials
