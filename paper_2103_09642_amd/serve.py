"""Serving loop over the C ABI: continuous batching of discharge cases.

Requests arrive over time (a Poisson stream), each asking for a number of RF
cycles of one discharge case.  A request is admitted when its device arena
(`edp_case_bytes`) fits the memory budget next to the resident cases, up to
the library's batch size.  Every iteration advances all resident cases
together by a fixed window of steps (each by at most what it still needs),
in one batch call, so that a short case leaves and a waiting one joins at
the next window boundary instead of waiting for the longest resident case.
Then it

* fails only the request whose case overflowed its particle capacity (its
  state is no longer physical; the others are untouched),
* gives a case whose plasma has grown past half of a capacity twice the
  room (`edp_case_resize`: the run continues bit for bit), within the
  request's capacity limit and the memory budget,
* retires the finished cases (counters and time-averaged densities).

A case's results do not depend on what it was batched with or when it was
resized: random numbers are keyed by particle identity and step, deposits
are integer sums, and every case keeps its own sort schedule.

Run as `python -m paper_2103_09642_amd.serve --rate 4 --duration 600`; it
prints one JSON line with offered and served load and p50/p99 time-to-result.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

WINDOW_STEPS = 4000   # steps per iteration (at most; a case takes what it still needs)
GROW_AT = 0.5         # fraction of a capacity in use that triggers a resize
MAX_RESIDENT = 256    # the library's largest batch


@dataclass
class Request:
    rid: int
    t_arrival: float              # seconds (wall clock) or iteration index (virtual clock)
    case: Dict
    cycles: int
    cap_limit: int = 0            # largest capacity per species the case may grow to (0: budget only)
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    steps_done: int = 0
    resizes: int = 0
    failed: str = ""
    result: Dict = field(default_factory=dict)

    @property
    def steps(self) -> int:
        return self.cycles * self.case["steps_per_cycle"]


def case_for(item: Dict, diag: bool = True, n_scale: float = 1.0) -> Dict:
    """The case of a stream item: a large-type case or batched-set case k,
    optionally with its particle count (and weight) rescaled.  Room for twice
    the seeded particles; the server grows it when the plasma does."""
    from . import workloads
    c = workloads.config_large() if item["kind"] == "large" else workloads.config_batch(item["case_k"])
    if n_scale != 1.0:
        n = max(256, int(c["n_init_e"] * n_scale))
        c = dict(c, weight=c["weight"] * c["n_init_e"] / n, n_init_e=n, n_init_i=n)
    if diag:
        c = dict(c, flags=list(c.get("flags", [])) + ["density"])
    return dict(c, cap_e=max(2 * c["n_init_e"], 1 << 16), cap_i=max(2 * c["n_init_i"], 1 << 16))


def offered_psteps(req: Request) -> float:
    """The work a request asks for at its seeded particle counts (electrons
    every step, ions every N_SUB-th)."""
    c = req.case
    return float(req.steps) * (c["n_init_e"] + c["n_init_i"] / c["ion_subcycle"])


class Server:
    """Admission + continuous batching over one context (one GPU stream)."""

    def __init__(self, ctx, budget_bytes: int, max_resident: int = MAX_RESIDENT, window: int = WINDOW_STEPS,
                 clock: Optional[Callable[[], float]] = None, grow: bool = True):
        self.ctx = ctx
        self.budget = int(budget_bytes)
        self.max_resident = max_resident
        self.window = window
        self.grow = grow
        self.clock = clock or time.perf_counter  # completion times; run() sets the origin
        self.waiting: List[Request] = []
        self.resident: List = []   # [Request, edupic.Case, bytes]
        self.used = 0
        self.done: List[Request] = []
        self.failed: List[Request] = []
        self.iterations = 0
        self.resizes = 0
        self.psteps = 0            # particle-steps of every request, finished or not

    def submit(self, req: Request):
        self.waiting.append(req)

    def _admit(self, now: float):
        keep = []
        for req in self.waiting:
            nbytes = self.ctx.case_bytes(req.case)
            if nbytes > self.budget:
                raise ValueError(f"request {req.rid} needs {nbytes} bytes, above the whole budget")
            if len(self.resident) < self.max_resident and self.used + nbytes <= self.budget:
                g = self.ctx.create_case(req.case)
                req.t_admit = now
                self.resident.append([req, g, nbytes])
                self.used += nbytes
            else:
                keep.append(req)
        self.waiting = keep

    def _maybe_grow(self, entry, k: Dict):
        req, g, nbytes = entry
        cap_e, cap_i = g.capacity()

        def target(n, cap):  # twice the room once half of it is in use
            if n <= GROW_AT * cap:
                return 0
            t = min(2 * cap, req.cap_limit) if req.cap_limit else 2 * cap
            return t if t > cap else 0
        want_e, want_i = target(k["n_e"], cap_e), target(k["n_i"], cap_i)
        if not (want_e or want_i):
            return
        grown = dict(req.case, cap_e=want_e or cap_e, cap_i=want_i or cap_i)
        more = self.ctx.case_bytes(grown)
        if self.used - nbytes + more > self.budget:
            return  # no room: the case runs on, and fails if it overflows
        g.resize(want_e, want_i)
        req.case = grown
        req.resizes += 1
        self.resizes += 1
        self.used += more - nbytes
        entry[2] = more

    def iterate(self, now: float) -> List[Request]:
        """Admit what fits, advance every resident case by one window,
        fail the overflowed, grow the crowded, retire the finished; returns
        the finished (and failed) requests."""
        self._admit(now)
        if not self.resident:
            return []
        steps = [min(self.window, req.steps - req.steps_done) for req, _, _ in self.resident]
        self.ctx.advance_steps([g for _, g, _ in self.resident], steps)
        self.iterations += 1
        finished, keep = [], []
        for entry, n in zip(self.resident, steps):
            req, g, nbytes = entry
            before = req.result.get("psteps", 0)
            k = g.counts()
            req.result["psteps"] = k["psteps_e"] + k["psteps_i"]
            self.psteps += req.result["psteps"] - before
            req.steps_done += n
            if k["overflow"]:
                req.failed = "capacity"
                req.result["counts"] = k
                g.destroy()
                self.used -= nbytes
                finished.append(req)
                continue
            if req.steps_done >= req.steps:
                ne, ni = g.density()
                req.result.update({"counts": k, "ne": ne, "ni": ni})
                g.destroy()
                self.used -= nbytes
                finished.append(req)
                continue
            if self.grow:
                self._maybe_grow(entry, k)
            keep.append(entry)
        self.resident = keep
        t = self.clock()
        for req in finished:
            req.t_done = t
            (self.failed if req.failed else self.done).append(req)
        return finished

    def run(self, requests: List[Request], virtual: bool = False, max_wall: float = 0.0,
            progress: float = 0.0) -> List[Request]:
        """Serve a stream.  Wall clock: requests become visible at their
        arrival time; with max_wall the loop stops after that many seconds,
        leaving the rest unserved; with progress a status line goes to stderr
        after an iteration at most every that many seconds.  Virtual clock
        (tests): arrival times are iteration numbers, so admission is
        deterministic."""
        pending = sorted(requests, key=lambda r: r.t_arrival)
        t0 = time.perf_counter()
        last = 0.0
        if not virtual:
            self.clock = lambda: time.perf_counter() - t0  # same origin as the arrival times
        it = 0
        while pending or self.waiting or self.resident:
            now = float(it) if virtual else time.perf_counter() - t0
            if max_wall and not virtual and now > max_wall:
                break
            while pending and pending[0].t_arrival <= now:
                self.submit(pending.pop(0))
            if not self.waiting and not self.resident:
                if virtual:
                    it += 1
                else:
                    time.sleep(max(0.0, min(0.05, pending[0].t_arrival - now)))
                continue
            self.iterate(now)
            it += 1
            if progress and not virtual:
                t = time.perf_counter() - t0
                if t - last >= progress:
                    last = t
                    print(f"[serve] {t:.0f} s: {len(requests) - len(pending)} arrived, {len(self.resident)} resident, "
                          f"{len(self.waiting)} waiting, {len(self.done)} done, {len(self.failed)} failed, "
                          f"{self.psteps / t:.3g} particle-steps/s served", file=sys.stderr, flush=True)
        self.unserved = pending + self.waiting + [e[0] for e in self.resident]
        return self.done


def latency_summary(reqs: List[Request]) -> Dict:
    lat = np.array([r.t_done - r.t_arrival for r in reqs])
    return {"n": int(lat.size), "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None}


def main(argv=None):
    ap = argparse.ArgumentParser(description="serve a Poisson stream of discharge cases on one GPU")
    ap.add_argument("--rate", type=float, default=4.0, help="arrivals per second")
    ap.add_argument("--duration", type=float, default=600.0, help="seconds of arrivals")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--p-large", type=float, default=0.1)
    ap.add_argument("--cyc-lo", type=int, default=20)
    ap.add_argument("--cyc-hi", type=int, default=200)
    ap.add_argument("--n-scale", type=float, default=1.0, help="scale every case's particle count")
    ap.add_argument("--budget-gb", type=float, default=0.0, help="memory budget (0: 80%% of the free HBM)")
    ap.add_argument("--mode", type=int, default=1, help="0 plain launches, 1 graphs")
    ap.add_argument("--window", type=int, default=WINDOW_STEPS, help="steps per iteration")
    ap.add_argument("--groups", type=int, default=0, help="lockstep groups (0: the library's default)")
    ap.add_argument("--small-max", type=int, default=0,
                    help="cases up to this many slots per species run in the persistent small-case kernel")
    ap.add_argument("--progress", type=float, default=30.0,
                    help="seconds between status lines on stderr (0: none)")
    ap.add_argument("--max-wall", type=float, default=0.0,
                    help="stop serving after this many seconds (0: until every request is done)")
    args = ap.parse_args(argv)

    import torch
    from . import edupic, workloads
    ctx = edupic.Context(0)
    ctx.set_xsec(workloads.synthetic_xsec())
    ctx.set_option(edupic.OPT_MODE, args.mode)
    if args.groups:
        ctx.set_option(edupic.OPT_GROUPS, args.groups)
    if args.small_max:
        ctx.set_option(edupic.OPT_SMALL_MAX, args.small_max)
    free, _ = torch.cuda.mem_get_info()
    budget = int(args.budget_gb * 2**30) if args.budget_gb > 0 else int(0.8 * free)
    stream = workloads.serving_stream(args.rate, args.duration, seed=args.seed, p_large=args.p_large,
                                      cyc_lo=args.cyc_lo, cyc_hi=args.cyc_hi)
    reqs = [Request(i, it["t_arrival"], case_for(it, n_scale=args.n_scale), it["cycles"])
            for i, it in enumerate(stream)]
    srv = Server(ctx, budget, window=args.window)
    t0 = time.perf_counter()
    done = srv.run(reqs, max_wall=args.max_wall, progress=args.progress)
    wall = time.perf_counter() - t0
    offered = sum(offered_psteps(r) for r in reqs) / args.duration
    out = {"requests": len(reqs), "completed": len(done), "failed": len(srv.failed),
           "unserved_at_stop": len(srv.unserved), "iterations": srv.iterations, "resizes": srv.resizes,
           "wall_s": round(wall, 3),
           "served_particle_steps_per_s": srv.psteps / wall,
           "offered_particle_steps_per_s": offered,
           "offered_note": "requested steps x seeded particles (ions every N_SUB-th step) over the arrival window",
           "latency": latency_summary(done),
           "stream": {"rate_hz": args.rate, "duration_s": args.duration, "p_large": args.p_large,
                      "cycles": [args.cyc_lo, args.cyc_hi], "n_scale": args.n_scale, "seed": args.seed,
                      "window_steps": args.window, "budget_gb": round(budget / 2**30, 1),
                      "max_wall_s": args.max_wall}}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
