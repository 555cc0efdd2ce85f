"""Benchmark of the PIC/MCC hot path on one MI355X.

Default workload (the largest single-GPU configuration): the batched
dual-frequency set -- 32 independent discharge cases (2.5 cm argon gap at
2.5-20 Pa / 350 K, 1000 grid nodes, V1 sin(2 pi 1.937 MHz t) with V1 in
100-400 V plus V2 sin(2 pi 27.12 MHz t) with V2 in 50-200 V, 2000 steps per
27.12 MHz period, each seeded as a uniform 1e15 m^-3 plasma of 1e6 electrons
+ 1e6 ions), advanced together by the batch runtime.  One benchmark "step" is
one 27.12 MHz period (2000 PIC/MCC time steps: field solve, push, walls,
collisions, births, deposit, periodic compaction/sort) of every case.  The
same line carries the plain single large case (1000 nodes, 8000 steps per
13.56 MHz period, 2e6 + 2e6 particles, with its time-averaged density and
EEPF diagnostics on and read every 10 RF cycles), so it reads "batched vs
plain".  Synthetic argon-like cross sections on 1e5 bins of 1 meV.

Other workloads: --workload large (the plain large case alone), batch64 (64
heterogeneous cases), small (the plain small case: 400 nodes, 4000 steps per
period, 1000 + 1000 seeds, 10 RF cycles, on the lockstep path and in the
persistent small-case kernel) and small256 (256 such cases, seeds 1..256).

Metric: particle-steps/s = (sum over steps of live electrons + sum over ion
steps of live ions) / wall time, inputs resident in HBM before the timed
region; the timed region runs in graph mode by default.  The roofline entry
is the electron kernel's (the dominant one): 48 algorithmic bytes per
electron step (read x, vx, vy, vz; write x, vx) times the electrons of a
launch over its mean duration, from HIP events on the library's stream
around every electron launch of a window of plain launches that continues
the same cases after the timed region (one lockstep group, so that no other
launch shares the chip; `--roof-same-groups` keeps the timed region's
groups); `step_frac` is the same 48 bytes per particle-step
over the whole timed region.  `traffic` is the counter-measured HBM bytes per
launch (committed summary) while the kernel source still matches the one
profiled.  The CPU baseline runs the single-threaded oracle, one case per
host core, on a bounded sample of the same workload.
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
HF_STEPS = 2000  # one 27.12 MHz period of the dual-frequency cases
MAX_CPU_WORKERS = 16  # the host-core share of one GPU
# a batch of cases also tries sorting every 400 steps (its windows are then
# longer than a graph holds, so it runs plain launches): the dual-frequency
# set ran 1% faster there than at 200
BATCH_SORT_EXTRA = 400


def measured_traffic(electrons_per_launch, workload):
    """HBM bytes per electron launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated with a copy kernel) of this
    workload, scaled to this run's electrons per launch; None when the kernel
    source has changed since the counters were taken or none were taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        with open(KERNEL_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    entry = t.get(workload)
    if not entry or entry.get("source_sha256") != sha:
        return None
    return round(entry["bytes_per_electron"] * electrons_per_launch)


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, MAX_CPU_WORKERS))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed benchmark steps (dual32: 27.12 MHz periods; large, batch64, small: RF cycles)")
    ap.add_argument("--warmup", type=int, default=2, help="untimed benchmark steps")
    ap.add_argument("--workload", choices=["dual32", "batch64", "large", "small", "small256"], default="dual32")
    ap.add_argument("--mode", type=int, default=-1, choices=(-1, 0, 1),
                    help="launch mode of the timed region: 0 plain, 1 graph windows; -1 (default) the "
                         "autotuner's choice for a batch of cases (several groups' graphs can overlap worse "
                         "than their plain launches), graph windows otherwise")
    ap.add_argument("--plain-steps", type=int, default=10,
                    help="dual32: timed RF cycles of the plain large case reported beside it (0: skip)")
    ap.add_argument("--cpu-steps", type=int, default=0,
                    help="oracle PIC steps per case for the CPU baseline (0: the workload's default)")
    ap.add_argument("--roof-same-groups", action="store_true",
                    help="time the roofline window in the timed region's lockstep groups (their launches "
                         "overlap, so each shares the chip) instead of one group")
    ap.add_argument("--roof-steps", type=int, default=0,
                    help="PIC steps of the profiled window (plain launches, HIP events per electron launch; "
                         "0: the workload's default)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--sort-every", type=int, default=0,
                    help="steps between compaction + cell sort; with --wg-per-cu and --groups "
                         "it fixes the schedule (default 0: the autotuner chooses on copies of the "
                         "workload's cases, outside the timed region)")
    ap.add_argument("--wg-per-cu", type=int, default=-1,
                    help="particle workgroups per CU (0: all that fit); -1: the autotuner's choice")
    ap.add_argument("--part-skew", type=int, default=-1,
                    help="per mille: the last dispatch layer's share of a case's chunks below the first's "
                         "(-1: the library's default)")
    ap.add_argument("--groups", type=int, default=0, choices=(0, 1, 2, 3, 4),
                    help="lockstep groups of a batched advance; 0: the autotuner's choice")
    ap.add_argument("--pic-steps", type=int, default=0,
                    help="profiling aid: time this many PIC steps instead of --steps benchmark steps")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="profiling aid: first copy a device buffer of this size (counter calibration)")
    ap.add_argument("--diag", action="store_true",
                    help="large: time-averaged density and EEPF on, read every 10 RF cycles (as the plain line)")
    ap.add_argument("--null-collision", action="store_true",
                    help="select colliding particles by the null-collision method")
    ap.add_argument("--sequential", action="store_true",
                    help="batched workloads: advance the cases one after another instead of as one batch")
    args = ap.parse_args()
    # the mode is tuned with the groups of a batch when the schedule is tuned
    args.tune_mode = args.mode == -1 and args.workload in ("dual32", "batch64") and not (
        args.sort_every and args.wg_per_cu >= 0 and args.groups)
    if args.mode == -1:
        args.mode = 1
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): independent cases shard "
              "across GPUs without communication, and one case's particles would need an int64 "
              "all-reduce of the deposit per step; neither is built here.", file=sys.stderr)
        sys.exit(2)

    # The CPU baseline first, in processes of its own, before this process
    # touches the GPU.
    cpu = None
    if not args.no_cpu:
        cpu = run_cpu_baseline(args)

    import torch
    from paper_2103_09642_amd import edupic, workloads  # noqa: F401

    if args.calib_copy_mb:
        a = torch.empty(args.calib_copy_mb << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload in ("small", "small256"):
        out = bench_small(args)
    elif args.workload == "large":
        out = bench_large(args)
    else:
        out = bench_batch(args)
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def run_cpu_baseline(args):
    if args.workload in ("dual32", "batch64"):
        dual = args.workload == "dual32"
        return cpu_baseline(batch_descs(args.workload), args.cpu_steps or (30 if dual else 40),
                            "dual-frequency set" if dual else "batched set")
    if args.workload == "large":
        return cpu_baseline([large_desc(args, False)], args.cpu_steps or 300, "plain large case")
    many = args.workload == "small256"
    return cpu_baseline(small_descs(args.workload), args.cpu_steps or (8000 if many else 40000),
                        "plain small case" + ("s" if many else ""))


# ---------------------------------------------------------------------------
# schedule
# ---------------------------------------------------------------------------

def choose_schedule(args, ctx, descs, warm):
    """The compaction + sort interval, the particle workgroups per CU and the
    lockstep groups: --sort-every, --wg-per-cu and --groups if all are given
    (a single case: the first two), else the autotuner's choice, made on
    copies of the workload's
    cases (created from the same seeded descriptors, advanced to the timed
    window's midpoint -- `warm(copies)` -- then tuned with every trial
    starting from that state, so that the trials see the regime of the timed
    window, and destroyed): the timed cases start from exactly the state they
    have without tuning.  Returns the tuning record."""
    from paper_2103_09642_amd import edupic, tune
    if len(descs) == 1 and not args.groups:
        args.groups = tune.DEFAULTS["groups"]  # no effect on a single case
    mode_candidates = (1, 0) if getattr(args, "tune_mode", False) else ()
    if args.sort_every and args.wg_per_cu >= 0 and args.groups:
        ctx.set_option(edupic.OPT_SORT_EVERY, args.sort_every)
        ctx.set_option(edupic.OPT_PART_WG_PER_CU, args.wg_per_cu)
        ctx.set_option(edupic.OPT_GROUPS, args.groups)
        return None
    t0 = time.perf_counter()
    copies = [ctx.create_case(d) for d in descs]

    def traced_measure(*a, **kw):
        # one line per trial on stderr, so that a long tuning stage shows progress
        t = tune.measure(*a, **kw)
        print(f"tuning trial: sort every {t.interval}, {t.wg_per_cu} workgroups per CU: {t.rate:.4g} "
              f"particle-steps/s", file=sys.stderr, flush=True)
        return t
    try:
        warm(copies)
        choice, trials = tune.tune_schedule(ctx, copies,
                                            candidates=(args.sort_every,) if args.sort_every else
                                            tune.DEFAULT_CANDIDATES + ((BATCH_SORT_EXTRA,) if len(descs) > 1
                                                                       else ()),
                                            wg_candidates=(args.wg_per_cu,) if args.wg_per_cu >= 0 else
                                            tune.DEFAULT_WG_CANDIDATES,
                                            restore_state=True,
                                            group_candidates=(args.groups,) if args.groups else
                                            tune.DEFAULT_GROUP_CANDIDATES,
                                            mode_candidates=mode_candidates, measure_fn=traced_measure)
    finally:
        for c in copies:
            c.destroy()
    args.sort_every, args.wg_per_cu = choice["sort_every"], choice["part_wg_per_cu"]
    args.groups = choice["groups"]
    if "mode" in choice:
        args.mode = choice["mode"]
    return {"seconds": round(time.perf_counter() - t0, 2),
            "on": "copies of the workload's cases advanced to the timed window's midpoint; "
                  "every trial starts from that state",
            "trials": [[t.interval, t.wg_per_cu, t.groups, t.mode, round(t.rate, 1)] for t in trials],
            "trial_fields": ["sort_every", "wg_per_cu", "groups", "mode (1 graph, 0 plain, -1 as set)",
                             "particle-steps/s"]}


# ---------------------------------------------------------------------------
# measurement helpers
# ---------------------------------------------------------------------------

def timed(ctx, cases, run):
    """Wall seconds of run() between device synchronisations and the
    particle-steps the cases' device counters gained meanwhile."""
    import torch
    ctx.sync()
    torch.cuda.synchronize()
    c0 = [g.counts() for g in cases]
    t0 = time.perf_counter()
    run()
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    c1 = [g.counts() for g in cases]
    pe = sum(b["psteps_e"] - a["psteps_e"] for a, b in zip(c0, c1))
    pi = sum(b["psteps_i"] - a["psteps_i"] for a, b in zip(c0, c1))
    return wall, pe, pi, c1


def roofline(ctx, cases, advance_steps, steps, workload, label, one_group=True):
    """Electron-kernel roofline from HIP events around every electron launch
    of `steps` PIC steps of plain launches (every case in one lockstep group,
    so that no other launch shares the chip, or the timed region's groups
    with one_group=False)."""
    from paper_2103_09642_amd import edupic
    ctx.set_option(edupic.OPT_MODE, 0)
    ctx.set_option(edupic.OPT_PROFILE, 1)
    groups_before = None
    if one_group and len(cases) > 1:
        groups_before = ctx_groups(ctx)
        ctx.set_option(edupic.OPT_GROUPS, 1)
    ctx.sync()
    ctx.read_profile()  # reset
    r0 = [g.counts() for g in cases]
    advance_steps(steps)
    ctx.sync()
    r1 = [g.counts() for g in cases]
    ms, launches = ctx.read_profile()
    ctx.set_option(edupic.OPT_PROFILE, 0)
    if groups_before:
        ctx.set_option(edupic.OPT_GROUPS, groups_before)
    if launches <= 0:
        return None
    avg_s = ms / 1e3 / launches
    epl = sum(b["psteps_e"] - a["psteps_e"] for a, b in zip(r0, r1)) / launches
    achieved = BYTES_PER_PSTEP * epl / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(epl, workload),
            "kernel": "k_particles<0> (electrons)", "avg_launch_us": round(avg_s * 1e6, 3),
            "electrons_per_launch": round(epl, 1), "launches": launches,
            "window": f"{steps} PIC steps of plain launches after the timed region, {label}"}


_GROUPS = {}


def ctx_groups(ctx):
    return _GROUPS.get(id(ctx), 2)


def set_groups(ctx, g):
    from paper_2103_09642_amd import edupic
    _GROUPS[id(ctx)] = g
    ctx.set_option(edupic.OPT_GROUPS, g)


def _oracle_sample(job):
    """Worker: seed one case in the oracle, then time `steps` PIC steps.
    Returns (particle-steps, seconds of stepping)."""
    case, steps = job
    from oracle import binding as orc
    from paper_2103_09642_amd.workloads import synthetic_xsec
    o = orc.Oracle(case, synthetic_xsec())
    o.seed()
    nsub = case["ion_subcycle"]
    pst, dtc = 0, 0.0
    for _ in range(steps):
        s = o.step_index
        pst += o.count(0) + (o.count(1) if s % nsub == 0 else 0)
        tc = time.perf_counter()
        o.step(1)
        dtc += time.perf_counter() - tc
    return pst, dtc


def cpu_baseline(descs, steps, what):
    """The oracle, one case per host core (at most MAX_CPU_WORKERS), each
    process seeding its case and timing `steps` PIC steps: the aggregate rate
    is the sum of the processes' own rates."""
    from multiprocessing import get_context
    cores = min(host_cores(), len(descs))
    jobs = [(d, steps) for d in descs[:cores]]
    t0 = time.perf_counter()
    with get_context("spawn").Pool(cores) as p:
        res = p.map(_oracle_sample, jobs)
    wall = time.perf_counter() - t0
    rate = sum(ps / dt for ps, dt in res if dt > 0)
    cpu_s = sum(dt for _, dt in res)
    return {"value": round(rate, 1), "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{what}: first {steps} PIC steps of {cores} of the workload's seeded cases, one "
                      f"single-threaded oracle process per core ({cpu_s:.1f} s of stepping, "
                      f"{wall:.1f} s wall with seeding)"}


def base_line(metric_value, wall, n_timed, args, config, roof, cpu, dtype="f64"):
    return {
        "metric": "particle-steps/s (push+MCC+deposit)",
        "value": round(metric_value, 1),
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / n_timed, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
        "roofline": roof,
        "cpu_baseline": cpu,
    }


def schedule_config(args, tuned):
    return {"mode": ["plain", "graph"][args.mode], "sort_every": args.sort_every, "wg_per_cu": args.wg_per_cu,
            "groups": args.groups, "schedule_tuning": tuned}


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def batch_descs(workload):
    from paper_2103_09642_amd import workloads
    xs = workloads.synthetic_xsec()
    descs = []
    if workload == "dual32":
        for k in range(1, 33):
            # run as given: the stability report, not the creation check, flags these
            c = workloads.config_dualfreq(k)
            descs.append(dict(c, flags=list(c.get("flags", [])) + ["allow_unstable"], cap_e=3 * c["n_init_e"],
                              cap_i=3 * c["n_init_i"]))
    else:
        for k in range(1, 65):
            c = workloads.config_batch(k, xs)
            # the high-pressure, high-voltage cases more than double their
            # seeded particle count within a few cycles: room for 8x
            descs.append(dict(c, cap_e=8 * c["n_init_e"], cap_i=8 * c["n_init_i"]))
    return descs


def bench_batch(args):
    """dual32: 32 dual-frequency cases, each advanced by one 27.12 MHz period
    (2000 steps) per benchmark step.  batch64: 64 heterogeneous cases, each
    advanced by one RF cycle of its own per benchmark step.  One batch call
    per timed region, or one call per case with --sequential."""
    from paper_2103_09642_amd import edupic, workloads
    dual = args.workload == "dual32"
    xs = workloads.synthetic_xsec()
    ctx = edupic.Context(0)
    if args.part_skew >= 0:
        ctx.set_option(edupic.OPT_PART_SKEW, args.part_skew)
    ctx.set_xsec(xs)
    ctx.set_option(edupic.OPT_MODE, args.mode)
    descs = batch_descs(args.workload)
    mid = args.warmup + args.steps // 2  # the timed window's midpoint, in benchmark steps

    def advance(cs, k):
        if dual:
            ctx.advance_steps(cs, [k * HF_STEPS] * len(cs))
        else:
            ctx.advance(cs, [k] * len(cs))

    tuned = choose_schedule(args, ctx, descs, lambda cs: advance(cs, mid))
    set_groups(ctx, args.groups)
    cases = [ctx.create_case(c) for c in descs]

    def run(k):
        if args.sequential:
            for g in cases:
                advance([g], k)
        else:
            advance(cases, k)

    if args.warmup:
        run(args.warmup)
    if args.pic_steps:
        wall, pe, pi, c1 = timed(ctx, cases, lambda: ctx.advance_steps(cases, [args.pic_steps] * len(cases)))
        n_timed = args.pic_steps / (HF_STEPS if dual else 1)
    else:
        wall, pe, pi, c1 = timed(ctx, cases, lambda: run(args.steps))
        n_timed = args.steps
    value = (pe + pi) / wall
    print(f"timed region: {wall:.3f} s, {pe} electron + {pi} ion particle-steps", file=sys.stderr, flush=True)
    roof = None
    if not args.no_profile:
        steps = args.roof_steps or (200 if dual else 400)
        roof = roofline(ctx, cases, lambda k: ctx.advance_steps(cases, [k] * len(cases)), steps, args.workload,
                        f"the same cases in the timed region's {ctx_groups(ctx)} lockstep group(s)"
                        if args.roof_same_groups else "all cases in one lockstep group",
                        one_group=not args.roof_same_groups)
        if roof:
            roof["step_frac"] = round(BYTES_PER_PSTEP * (pe + pi) / wall / 1e9 / HBM_PEAK_GBS, 4)
    for g in cases:
        g.destroy()
    ctx.close()
    cpu = None
    config = {"workload": ("batched dual-frequency set: 32 cases (2.5-20 Pa, 100-400 V at 1.937 MHz + 50-200 V "
                           "at 27.12 MHz, 2.5 cm, 1000 nodes, 1e6+1e6 particles each); step = one 27.12 MHz "
                           "period (2000 PIC steps) of every case") if dual else
                          ("batched set: 64 heterogeneous cases (5-100 Pa, 100-500 V, 1.5-5 cm, 200-1000 nodes, "
                           "1e4-5e5 particles per species); step = 1 RF cycle of every case"),
              "execution": "sequential" if args.sequential else "one batch",
              **schedule_config(args, tuned),
              "electron_psteps": pe, "ion_psteps": pi,
              "particles_live_end": sum(c["n_e"] + c["n_i"] for c in c1)}
    out = base_line(value, wall, n_timed, args, config, roof, cpu)
    if dual and args.plain_steps > 0 and not args.sequential:
        out["plain"] = plain_large(args)
    return out


def large_desc(args, diag):
    from paper_2103_09642_amd import workloads
    case = workloads.config_large()
    flags = list(case["flags"])
    if args.null_collision:
        flags.append("null_collision")
    if diag:
        flags += ["density", "eepf"]
    return dict(case, flags=flags)


def run_large(args, cycles, warmup, diag, tune_on):
    """The plain large case: tuned (or fixed) schedule, `warmup` untimed then
    `cycles` timed RF cycles; with diag the time-averaged density and EEPF
    are read (and restarted) every 10 cycles inside the timed region."""
    from paper_2103_09642_amd import edupic, workloads
    case = large_desc(args, diag)
    ctx = edupic.Context(0)
    if args.part_skew >= 0:
        ctx.set_option(edupic.OPT_PART_SKEW, args.part_skew)
    ctx.set_xsec(workloads.synthetic_xsec())
    ctx.set_option(edupic.OPT_MODE, args.mode)
    mid = warmup + cycles // 2
    tuned = choose_schedule(tune_on, ctx, [case], lambda cs: ctx.advance(cs, [mid] * len(cs)))
    g = ctx.create_case(case)
    if warmup:
        g.advance(warmup)

    def run():
        left = cycles
        while left > 0:
            k = min(10, left) if diag else left
            g.advance(k)
            left -= k
            if diag and k == 10:
                g.density(reset=False)
                g.eepf(reset=True)

    wall, pe, pi, c1 = timed(ctx, [g], run)
    return ctx, g, case, tuned, wall, pe, pi, c1


def plain_large(args):
    """The plain large case beside a batched line: its own tuned schedule,
    density and EEPF on."""
    class A:  # the tuner's inputs for this case alone
        sort_every, wg_per_cu, groups = 0, -1, 0
    ctx, g, case, tuned, wall, pe, pi, c1 = run_large(args, args.plain_steps, 1, True, A)
    g.destroy()
    ctx.close()
    return {"workload": "plain large single case: 1000 nodes, 8000 steps/RF cycle, 2e6+2e6 seeded uniform "
                        "1e15 m^-3, 10 Pa Ar, 250 V 13.56 MHz, time-averaged density and EEPF read every 10 "
                        "cycles",
            "value": round((pe + pi) / wall, 1), "unit": "particle-steps/s", "rf_cycles": args.plain_steps,
            "ms_per_rf_cycle": round(wall * 1e3 / args.plain_steps, 3),
            "schedule": [A.sort_every, A.wg_per_cu], "tuning_seconds": tuned and tuned["seconds"]}


def bench_large(args):
    ctx, g, case, tuned, wall, pe, pi, c1 = run_large(args, args.steps if not args.pic_steps else 0,
                                                       args.warmup, args.diag, args)
    if args.pic_steps:
        wall, pe, pi, c1 = timed(ctx, [g], lambda: g.advance_steps(args.pic_steps))
    print(f"timed region: {wall:.3f} s, {pe} electron + {pi} ion particle-steps", file=sys.stderr, flush=True)
    value = (pe + pi) / wall
    roof = None
    if not args.no_profile:
        roof = roofline(ctx, [g], g.advance_steps, args.roof_steps or 1000, "large", "the same case")
        if roof:
            roof["step_frac"] = round(BYTES_PER_PSTEP * (pe + pi) / wall / 1e9 / HBM_PEAK_GBS, 4)
    g.destroy()
    ctx.close()
    cpu = None
    n_timed = args.steps if not args.pic_steps else args.pic_steps / case["steps_per_cycle"]
    config = {"workload": "plain large single case: 1000 nodes, 8000 steps/RF cycle, 2e6+2e6 seeded uniform "
                          "1e15 m^-3, 10 Pa Ar, 250 V 13.56 MHz; step = 1 RF cycle",
              "collision_selection": "null collision" if args.null_collision else "direct",
              "diagnostics": "time-averaged density and EEPF, read every 10 RF cycles" if args.diag else "none",
              **schedule_config(args, tuned),
              "electrons_live_end": c1[0]["n_e"], "ions_live_end": c1[0]["n_i"],
              "electron_psteps": pe, "ion_psteps": pi}
    return base_line(value, wall, n_timed, args, config, roof, cpu)


def small_descs(workload):
    from paper_2103_09642_amd import workloads
    n = 256 if workload == "small256" else 1
    return [workloads.base_case(seed=k, cap_e=1 << 16, cap_i=1 << 16) for k in range(1, n + 1)]


def bench_small(args):
    """The plain small case (400 nodes, 4000 steps per period, 1000 + 1000
    seeds, seed 1) for --steps RF cycles, or 256 such cases (seeds 1..256):
    on the lockstep path and in the persistent small-case kernel (one
    workgroup per case for the whole window); the line's value is the faster
    of the two, both are reported with their time-to-result."""
    from paper_2103_09642_amd import edupic, workloads
    many = args.workload == "small256"
    descs = small_descs(args.workload)
    xs = workloads.synthetic_xsec()
    res = {}
    for path, small_max in (("lockstep", 0), ("persistent", 1 << 30)):
        ctx = edupic.Context(0)
        if args.part_skew >= 0:
            ctx.set_option(edupic.OPT_PART_SKEW, args.part_skew)
        ctx.set_xsec(xs)
        ctx.set_option(edupic.OPT_MODE, args.mode)
        ctx.set_option(edupic.OPT_SORT_EVERY, args.sort_every or 100)
        ctx.set_option(edupic.OPT_SMALL_MAX, small_max)
        if args.groups:
            ctx.set_option(edupic.OPT_GROUPS, args.groups)
        cases = [ctx.create_case(d) for d in descs]
        if args.warmup:
            ctx.advance(cases, [args.warmup] * len(cases))
        wall, pe, pi, c1 = timed(ctx, cases, lambda: ctx.advance(cases, [args.steps] * len(cases)))
        res[path] = {"value": round((pe + pi) / wall, 1), "seconds": round(wall, 4),
                     "ms_per_rf_cycle": round(wall * 1e3 / args.steps, 3), "electron_psteps": pe,
                     "ion_psteps": pi, "particles_live_end": sum(c["n_e"] + c["n_i"] for c in c1)}
        print(f"{path}: {wall:.3f} s, {pe} + {pi} particle-steps", file=sys.stderr, flush=True)
        for g in cases:
            g.destroy()
        ctx.close()
    best = max(res, key=lambda k: res[k]["value"])
    cpu = None
    config = {"workload": ("256 plain small cases (seeds 1..256)" if many else "plain small case (seed 1)") +
                          ": 2.5 cm, 10 Pa, 400 nodes, 4000 steps/RF cycle, 250 V 13.56 MHz, 1000+1000 "
                          "seeded, W 3.5e5; step = 1 RF cycle of every case; latency-bound, not a roofline "
                          "configuration",
              "mode": ["plain", "graph"][args.mode], "paths": res, "reported_path": best}
    return base_line(res[best]["value"], res[best]["seconds"], args.steps, args, config, None, cpu)


if __name__ == "__main__":
    main()
