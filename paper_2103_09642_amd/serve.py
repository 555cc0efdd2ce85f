"""Serving loop over the C ABI: continuous batching of discharge cases.

Requests arrive over time (a Poisson stream), each asking for a number of RF
cycles of one discharge case.  A request is admitted when its device arena
(`edp_case_bytes`) fits the memory budget next to the resident cases; all
resident cases then advance together.  Every iteration advances each of them
by one RF cycle of its own in a single lockstep batch call (one launch per
kernel per step for the whole batch), retires the cases that are done
(reading their counters and time-averaged densities) and admits new
arrivals.  A case's results do not depend on what it was batched with:
random numbers are keyed by particle identity and step, deposits are integer
sums, and every case keeps its own sort schedule.

Run as `python -m paper_2103_09642_amd.serve --rate 2 --duration 30`; it
prints one JSON line with offered and served load and p50/p99 latency.
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    t_arrival: float              # seconds (wall clock) or iteration index (virtual clock)
    case: Dict
    cycles: int
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    cycles_done: int = 0
    result: Dict = field(default_factory=dict)


def case_for(item: Dict, diag: bool = True, n_scale: float = 1.0) -> Dict:
    """The case of a stream item: a large-type case or batched-set case k,
    optionally with its particle count (and weight) rescaled."""
    from . import workloads
    c = workloads.config_large() if item["kind"] == "large" else workloads.config_batch(item["case_k"])
    if n_scale != 1.0:
        n = max(256, int(c["n_init_e"] * n_scale))
        c = dict(c, weight=c["weight"] * c["n_init_e"] / n, n_init_e=n, n_init_i=n)
    if diag:
        c = dict(c, flags=list(c.get("flags", [])) + ["density"])
    # room for growth: strongly ionizing cases more than double within a few cycles
    return dict(c, cap_e=max(8 * c["n_init_e"], 1 << 18), cap_i=max(8 * c["n_init_i"], 1 << 18))


class Server:
    """Admission + continuous batching over one context (one GPU stream)."""

    def __init__(self, ctx, budget_bytes: int, max_resident: int = 256,
                 clock: Optional[Callable[[], float]] = None):
        self.ctx = ctx
        self.budget = int(budget_bytes)
        self.max_resident = max_resident
        self.clock = clock or time.perf_counter  # completion times; run() sets the origin
        self.waiting: List[Request] = []
        self.resident: List = []   # (Request, edupic.Case, bytes)
        self.used = 0
        self.done: List[Request] = []
        self.iterations = 0

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
                self.resident.append((req, g, nbytes))
                self.used += nbytes
            else:
                keep.append(req)
        self.waiting = keep

    def iterate(self, now: float) -> List[Request]:
        """Admit what fits, advance every resident case by one RF cycle,
        retire the finished ones; returns them."""
        self._admit(now)
        if not self.resident:
            return []
        self.ctx.advance([g for _, g, _ in self.resident], [1] * len(self.resident))
        self.iterations += 1
        finished, keep = [], []
        for req, g, nbytes in self.resident:
            req.cycles_done += 1
            if req.cycles_done >= req.cycles:
                ne, ni = g.density()
                req.result = {"counts": g.counts(), "ne": ne, "ni": ni}
                g.destroy()
                self.used -= nbytes
                finished.append(req)
            else:
                keep.append((req, g, nbytes))
        self.resident = keep
        t = self.clock()
        for req in finished:
            req.t_done = t
        self.done.extend(finished)
        return finished

    def run(self, requests: List[Request], virtual: bool = False) -> List[Request]:
        """Serve a stream.  Wall clock: requests become visible at their
        arrival time.  Virtual clock (tests): arrival times are iteration
        numbers, so admission is deterministic."""
        pending = sorted(requests, key=lambda r: r.t_arrival)
        t0 = time.perf_counter()
        if not virtual:
            self.clock = lambda: time.perf_counter() - t0  # same origin as the arrival times
        it = 0
        while pending or self.waiting or self.resident:
            now = float(it) if virtual else time.perf_counter() - t0
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
        return self.done


def latency_summary(reqs: List[Request]) -> Dict:
    lat = np.array([r.t_done - r.t_arrival for r in reqs])
    return {"n": int(lat.size), "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None}


def main(argv=None):
    ap = argparse.ArgumentParser(description="serve a Poisson stream of discharge cases on one GPU")
    ap.add_argument("--rate", type=float, default=2.0, help="arrivals per second")
    ap.add_argument("--duration", type=float, default=30.0, help="seconds of arrivals")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--p-large", type=float, default=0.1)
    ap.add_argument("--cyc-lo", type=int, default=2)
    ap.add_argument("--cyc-hi", type=int, default=20)
    ap.add_argument("--n-scale", type=float, default=1.0, help="scale every case's particle count")
    ap.add_argument("--budget-gb", type=float, default=128.0)
    ap.add_argument("--mode", type=int, default=1, help="0 plain launches, 1 graphs")
    args = ap.parse_args(argv)

    from . import edupic, workloads
    ctx = edupic.Context(0)
    ctx.set_xsec(workloads.synthetic_xsec())
    ctx.set_option(edupic.OPT_MODE, args.mode)
    stream = workloads.serving_stream(args.rate, args.duration, seed=args.seed, p_large=args.p_large,
                                      cyc_lo=args.cyc_lo, cyc_hi=args.cyc_hi)
    reqs = [Request(i, it["t_arrival"], case_for(it, n_scale=args.n_scale), it["cycles"])
            for i, it in enumerate(stream)]
    srv = Server(ctx, int(args.budget_gb * 2**30))
    t0 = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t0
    psteps = sum(r.result["counts"]["psteps_e"] + r.result["counts"]["psteps_i"] for r in done)
    # offered load: the work of every request, spread over the arrival window
    out = {"requests": len(done), "iterations": srv.iterations, "wall_s": round(wall, 3),
           "served_particle_steps_per_s": psteps / wall,
           "offered_particle_steps_per_s": psteps / args.duration,
           "latency": latency_summary(done),
           "stream": {"rate_hz": args.rate, "duration_s": args.duration, "p_large": args.p_large,
                      "cycles": [args.cyc_lo, args.cyc_hi], "n_scale": args.n_scale, "seed": args.seed}}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
