"""Benchmark of the PIC/MCC hot path on one MI355X.

Workload: the plain large single case -- 2.5 cm argon gap at 10 Pa / 350 K,
1000 grid nodes, 8000 steps per 13.56 MHz period, 250 V sine, started from a
uniform 1e15 m^-3 plasma seeded as 2e6 electrons + 2e6 ions (W = 1250),
synthetic argon-like cross sections on 1e5 bins of 1 meV.  One benchmark
"step" is one RF cycle (8000 PIC/MCC time steps: field solve, push, walls,
collisions, births, deposit, periodic compaction/sort).

Metric: particle-steps/s = (sum over steps of live electrons + sum over ion
steps of live ions) / wall time, inputs resident in HBM before the timed
region.  The timed region runs in graph mode by default.  The roofline entry uses the
electron kernel (the dominant one): 48 algorithmic bytes per electron step
(read x, vx, vy, vz; write x, vx) divided by its mean launch time, from HIP
events on the library's stream around every electron launch of a window of
plain launches that continues the same case after the timed region; its
`traffic` is the counter-measured HBM bytes per launch (committed summary)
while the kernel source still matches the one profiled.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_particles_electrons_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2103_09642_amd", "csrc", "kernels.hip")


def measured_traffic(electrons_per_launch):
    """HBM bytes per electron launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated with a copy kernel), scaled to this
    run's electrons per launch; None when the kernel source has changed since
    the counters were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != sha:
        return None
    return round(t["bytes_per_electron"] * electrons_per_launch)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed RF cycles")
    ap.add_argument("--warmup", type=int, default=2, help="untimed RF cycles")
    ap.add_argument("--mode", type=int, default=1, help="launch mode of the timed region: 0 plain, 1 graph")
    ap.add_argument("--cpu-steps", type=int, default=300, help="oracle PIC steps for the CPU baseline")
    ap.add_argument("--roof-steps", type=int, default=1000,
                    help="PIC steps of the profiled window (plain launches, HIP events per electron launch)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--sort-every", type=int, default=0,
                    help="steps between compaction + cell sort; with --wg-per-cu and --apply-lanes it "
                         "fixes the schedule "
                         "(default 0: the autotuner chooses both on copies of the workload's cases, "
                         "outside the timed region)")
    ap.add_argument("--wg-per-cu", type=int, default=-1,
                    help="particle workgroups per CU (0: all that fit); -1: the autotuner's choice")
    ap.add_argument("--apply-lanes", type=int, default=0,
                    help="lanes per event list in the head (16, 32, 64); 0: the autotuner's choice")
    ap.add_argument("--groups", type=int, default=0, choices=(0, 1, 2, 3, 4),
                    help="lockstep groups of a batched advance, each on a stream of its own "
                         "(batch64/dual32; a single case runs alone); 0: the autotuner's choice")
    ap.add_argument("--pic-steps", type=int, default=0,
                    help="profiling aid: time this many PIC steps instead of --steps RF cycles")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="profiling aid: first copy a device buffer of this size (counter calibration)")
    ap.add_argument("--workload", choices=["large", "batch64", "dual32"], default="large",
                    help="large: the single 2e6+2e6 case (default); batch64: the 64-case heterogeneous set")
    ap.add_argument("--null-collision", action="store_true",
                    help="select colliding particles by the null-collision method")
    ap.add_argument("--sequential", action="store_true",
                    help="batch64 only: advance the cases one after another instead of as one batch")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): independent cases shard "
              "across GPUs without communication, and one case's particles would need an int64 "
              "all-reduce of the deposit per step; neither is built here.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2103_09642_amd import edupic, workloads

    if args.workload in ("batch64", "dual32"):
        return bench_batch(args)

    case = workloads.config_large()
    if args.null_collision:
        case = dict(case, flags=list(case["flags"]) + ["null_collision"])
    xs = workloads.synthetic_xsec()
    ctx = edupic.Context(0)
    ctx.set_xsec(xs)
    ctx.set_option(edupic.OPT_MODE, args.mode)
    ctx.set_option(edupic.OPT_PROFILE, 0)
    if args.calib_copy_mb:
        a = torch.empty(args.calib_copy_mb << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    mid = args.warmup + args.steps // 2  # the timed window's midpoint, in RF cycles
    tuned = choose_schedule(args, ctx, [case], lambda cs: ctx.advance(cs, [mid] * len(cs)))
    g = ctx.create_case(case)
    if args.warmup:
        g.advance(args.warmup)
    ctx.sync()
    torch.cuda.synchronize()
    c0 = g.counts()
    t0 = time.perf_counter()
    if args.pic_steps:
        g.advance_steps(args.pic_steps)
    else:
        g.advance(args.steps)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c1 = g.counts()
    wall = t1 - t0
    pe = c1["psteps_e"] - c0["psteps_e"]
    pi = c1["psteps_i"] - c0["psteps_i"]
    value = (pe + pi) / wall
    print(f"timed region: {wall:.3f} s, {pe} electron + {pi} ion particle-steps, mode {args.mode}",
          file=sys.stderr, flush=True)

    # Roofline of the dominant kernel: HIP events around every electron launch
    # of a window of plain launches continuing the same case.
    roof = None
    if not args.no_profile and args.roof_steps > 0:
        ctx.set_option(edupic.OPT_MODE, 0)
        ctx.set_option(edupic.OPT_PROFILE, 1)
        ctx.sync()
        ctx.read_profile()  # reset
        r0 = g.counts()
        g.advance_steps(args.roof_steps)
        ctx.sync()
        r1 = g.counts()
        ms, launches = ctx.read_profile()
        ctx.set_option(edupic.OPT_PROFILE, 0)
        if launches > 0:
            avg_s = ms / 1e3 / launches
            epl = (r1["psteps_e"] - r0["psteps_e"]) / launches
            achieved = BYTES_PER_PSTEP * epl / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(epl),
                    "kernel": "k_particles<0> (electrons)", "avg_launch_us": round(avg_s * 1e6, 3),
                    "electrons_per_launch": round(epl, 1), "launches": launches,
                    "window": f"{args.roof_steps} PIC steps of plain launches after the timed region"}
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
    n_timed = args.steps if not args.pic_steps else args.pic_steps / case["steps_per_cycle"]
    out = {
        "metric": "particle-steps/s (push+MCC+deposit)",
        "value": round(value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / n_timed, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plain large single case: 1000 nodes, 8000 steps/RF cycle, 2e6+2e6 "
                               "seeded uniform 1e15 m^-3, 10 Pa Ar, 250 V 13.56 MHz; step = 1 RF cycle",
                   "mode": ["plain", "graph"][args.mode], "collision_selection":
                       "null collision" if args.null_collision else "direct", "sort_every": args.sort_every,
                   "wg_per_cu": args.wg_per_cu, "apply_lanes": args.apply_lanes, "schedule_tuning": tuned,
                   "electrons_live_end": c1["n_e"],
                   "ions_live_end": c1["n_i"], "electron_psteps": pe, "ion_psteps": pi},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def choose_schedule(args, ctx, descs, warm):
    """The compaction + sort interval, the particle workgroups per CU, the
    lanes per event list and the lockstep groups: --sort-every, --wg-per-cu,
    --apply-lanes and --groups if all are given (a single case: the first
    three), else the autotuner's choice, made on copies of the
    workload's cases (created from the same seeded descriptors, advanced to
    the timed window's midpoint -- `warm(copies)` -- then tuned with every
    trial starting from that state, so that the trials see the regime of the
    timed window, and destroyed): the timed cases start from exactly the
    state they have without tuning.  Returns the tuning record."""
    from paper_2103_09642_amd import edupic, tune
    if len(descs) == 1 and not args.groups:
        args.groups = tune.DEFAULTS["groups"]  # no effect on a single case
    if args.sort_every and args.wg_per_cu >= 0 and args.apply_lanes and args.groups:
        ctx.set_option(edupic.OPT_SORT_EVERY, args.sort_every)
        ctx.set_option(edupic.OPT_PART_WG_PER_CU, args.wg_per_cu)
        ctx.set_option(edupic.OPT_APPLY_LANES, args.apply_lanes)
        ctx.set_option(edupic.OPT_GROUPS, args.groups)
        return None
    t0 = time.perf_counter()
    copies = [ctx.create_case(d) for d in descs]
    try:
        warm(copies)
        choice, trials = tune.tune_schedule(ctx, copies,
                                            candidates=(args.sort_every,) if args.sort_every else
                                            tune.DEFAULT_CANDIDATES,
                                            wg_candidates=(args.wg_per_cu,) if args.wg_per_cu >= 0 else
                                            tune.DEFAULT_WG_CANDIDATES,
                                            lane_candidates=(args.apply_lanes,) if args.apply_lanes else
                                            tune.DEFAULT_LANE_CANDIDATES, restore_state=True,
                                            group_candidates=(args.groups,) if args.groups else
                                            tune.DEFAULT_GROUP_CANDIDATES)
    finally:
        for c in copies:
            c.destroy()
    args.sort_every, args.wg_per_cu = choice["sort_every"], choice["part_wg_per_cu"]
    args.apply_lanes, args.groups = choice["apply_lanes"], choice["groups"]
    return {"seconds": round(time.perf_counter() - t0, 2),
            "on": "copies of the workload's cases advanced to the timed window's midpoint; "
                  "every trial starts from that state",
            "trials": [[t.interval, t.wg_per_cu, t.lanes, t.groups, round(t.rate, 1)] for t in trials],
            "trial_fields": ["sort_every", "wg_per_cu", "apply_lanes", "groups", "particle-steps/s"]}


def bench_batch(args):
    """batch64: 64 heterogeneous cases (pressure, voltage, gap, grid, particle
    count and N_t all differ), each advanced by RF cycles of its own.
    dual32: 32 dual-frequency cases (1.937 + 27.12 MHz, 1e6 per species,
    1000 nodes), each advanced by one 27.12 MHz period (2000 steps) per
    benchmark step.  One batch call per timed region, or one call per case
    with --sequential."""
    import torch
    from paper_2103_09642_amd import edupic, workloads

    xs = workloads.synthetic_xsec()
    ctx = edupic.Context(0)
    ctx.set_xsec(xs)
    ctx.set_option(edupic.OPT_MODE, args.mode)
    # the high-pressure, high-voltage cases more than double their seeded
    # particle count within a few cycles: room for 8x
    descs = []
    dual = args.workload == "dual32"
    for k in range(1, 33 if dual else 65):
        if dual:
            # run as given: the stability report, not the creation check, flags these
            c = workloads.config_dualfreq(k)
            c = dict(c, flags=list(c.get("flags", [])) + ["allow_unstable"], cap_e=3 * c["n_init_e"],
                     cap_i=3 * c["n_init_i"])
        else:
            c = workloads.config_batch(k, xs)
            c = dict(c, cap_e=8 * c["n_init_e"], cap_i=8 * c["n_init_i"])
        descs.append(c)
    hf_steps = 2000  # one 27.12 MHz period of the dual-frequency cases

    mid = args.warmup + args.steps // 2  # the timed window's midpoint, in benchmark steps

    def warm(cs):
        if dual:
            ctx.advance_steps(cs, [mid * hf_steps] * len(cs))
        else:
            ctx.advance(cs, [mid] * len(cs))
    tuned = choose_schedule(args, ctx, descs, warm)
    cases = [ctx.create_case(c) for c in descs]

    def run(cycles):
        if args.sequential:
            for g in cases:
                if dual:
                    g.advance_steps(cycles * hf_steps)
                else:
                    g.advance(cycles)
        elif dual:
            ctx.advance_steps(cases, [cycles * hf_steps] * len(cases))
        else:
            ctx.advance(cases, [cycles] * len(cases))

    if args.warmup:
        run(args.warmup)
    ctx.sync()
    torch.cuda.synchronize()
    c0 = [g.counts() for g in cases]
    t0 = time.perf_counter()
    run(args.steps)
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = [g.counts() for g in cases]
    ps = sum(b["psteps_e"] - a["psteps_e"] + b["psteps_i"] - a["psteps_i"] for a, b in zip(c0, c1))
    out = {
        "metric": "particle-steps/s (push+MCC+deposit)",
        "value": round(ps / wall, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("batched dual-frequency set: 32 cases (2.5-20 Pa, 100-400 V at 1.937 MHz + "
                                "50-200 V at 27.12 MHz, 2.5 cm, 1000 nodes, 1e6+1e6 particles each); "
                                "step = one 27.12 MHz period (2000 PIC steps) of every case") if dual else
                               ("batched set: 64 heterogeneous cases (5-100 Pa, 100-500 V, 1.5-5 cm, "
                                "200-1000 nodes, 1e4-5e5 particles per species); step = 1 RF cycle of every case"),
                   "mode": ["plain", "graph"][args.mode],
                   "execution": "sequential" if args.sequential else "one batch",
                   "groups": args.groups,
                   "sort_every": args.sort_every, "wg_per_cu": args.wg_per_cu, "apply_lanes": args.apply_lanes,
                   "schedule_tuning": tuned,
                   "particle_steps": ps,
                   "particles_live_end": sum(c["n_e"] + c["n_i"] for c in c1)},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
