"""Benchmark of the PIC/MCC hot path on one MI355X.

Workload: the plain large single case -- 2.5 cm argon gap at 10 Pa / 350 K,
1000 grid nodes, 8000 steps per 13.56 MHz period, 250 V sine, started from a
uniform 1e15 m^-3 plasma seeded as 2e6 electrons + 2e6 ions (W = 1250),
synthetic argon-like cross sections on 1e5 bins of 1 meV.  One benchmark
"step" is one RF cycle (8000 PIC/MCC time steps: field solve, push, walls,
collisions, births, deposit, periodic compaction/sort).

Metric: particle-steps/s = (sum over steps of live electrons + sum over ion
steps of live ions) / wall time, inputs resident in HBM before the timed
region.  The roofline entry uses the electron kernel (the dominant one):
48 algorithmic bytes per electron step (read x, vx, vy, vz; write x, vx)
divided by its mean launch time from HIP events on the library's stream.
The CPU baseline runs the single-threaded oracle on a bounded sample of the
same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_PSTEP = 48


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed RF cycles")
    ap.add_argument("--warmup", type=int, default=2, help="untimed RF cycles")
    ap.add_argument("--mode", type=int, default=-1, help="0 plain, 1 graph (default: best)")
    ap.add_argument("--cpu-steps", type=int, default=60, help="oracle PIC steps for the CPU baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--sort-every", type=int, default=100, help="steps between compaction + cell sort")
    ap.add_argument("--pic-steps", type=int, default=0,
                    help="profiling aid: time this many PIC steps instead of --steps RF cycles")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="profiling aid: first copy a device buffer of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): independent cases shard "
              "across GPUs without communication, and one case's particles would need an int64 "
              "all-reduce of the deposit per step; neither is built here.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2103_09642_amd import edupic, workloads

    case = workloads.config_large()
    xs = workloads.synthetic_xsec()
    ctx = edupic.Context(0)
    ctx.set_xsec(xs)
    mode = 0 if args.mode < 0 else args.mode
    ctx.set_option(edupic.OPT_MODE, mode)
    ctx.set_option(edupic.OPT_SORT_EVERY, args.sort_every)
    profile = not args.no_profile and mode == 0
    ctx.set_option(edupic.OPT_PROFILE, 1 if profile else 0)
    if args.calib_copy_mb:
        a = torch.empty(args.calib_copy_mb << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    g = ctx.create_case(case)
    if args.warmup:
        g.advance(args.warmup)
    ctx.sync()
    c0 = g.counts()
    ctx.read_profile()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.pic_steps:
        g.advance_steps(args.pic_steps)
    else:
        g.advance(args.steps)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = g.counts()
    ms, launches = ctx.read_profile()
    wall = t1 - t0
    pe = c1["psteps_e"] - c0["psteps_e"]
    pi = c1["psteps_i"] - c0["psteps_i"]
    value = (pe + pi) / wall
    roof = None
    if profile and launches > 0:
        avg_s = ms / 1e3 / launches
        bytes_per_launch = BYTES_PER_PSTEP * pe / launches
        achieved = bytes_per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_particles<electrons>", "avg_launch_us": round(avg_s * 1e6, 3),
                "electrons_per_launch": round(pe / launches, 1)}
    cpu = None
    if not args.no_cpu:
        from oracle import binding as orc
        o = orc.Oracle(case, xs)
        o.seed()
        nsub = case["ion_subcycle"]
        pst, n_ion_steps, dtc = 0, 0, 0.0
        for _ in range(args.cpu_steps):
            s = o.step_index
            pst += o.count(0)
            if s % nsub == 0:
                pst += o.count(1)
                n_ion_steps += 1
            tc = time.perf_counter()
            o.step(1)
            dtc += time.perf_counter() - tc
        cpu = {"value": round(pst / dtc, 1), "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
               "sample": f"first {args.cpu_steps} PIC steps of the same seeded workload "
                         f"({case['n_init_e']}+{case['n_init_i']} particles, {n_ion_steps} ion steps), "
                         f"single thread, {dtc:.1f} s"}
    out = {
        "metric": "particle-steps/s (push+MCC+deposit)",
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / (args.steps if not args.pic_steps else args.pic_steps / case["steps_per_cycle"]), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plain large single case: 1000 nodes, 8000 steps/RF cycle, 2e6+2e6 "
                               "seeded uniform 1e15 m^-3, 10 Pa Ar, 250 V 13.56 MHz; step = 1 RF cycle",
                   "mode": ["plain", "graph"][mode], "electrons_live_end": c1["n_e"], "ions_live_end": c1["n_i"],
                   "electron_psteps": pe, "ion_psteps": pi},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
