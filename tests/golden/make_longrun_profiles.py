"""Write tests/golden/longrun_c1_profiles.json: the oracle's time-averaged
profiles for the long-run statistical parity test.

The case is the small plain case's geometry and gas (2.5 cm, 10 Pa argon at
350 K, 400 nodes, 4000 steps per 13.56 MHz period, 250 V, N_SUB = 20, the
synthetic cross sections), seeded with N0 electrons + N0 ions.  For every
seed the oracle runs WARM RF cycles, restarts its diagnostics and runs
MEASURE more with the time-averaged density and mean-energy diagnostics of
section 3.5 on; the profiles n_e(x), n_i(x) and <eps_e>(x) of each seed are
stored, with the spread of the seeds about their mean: the relative L2
distance of each seed's profile from the mean over the seeds, over the nodes
where the mean n_e is at least 10% of its maximum.

This script calls only the oracle (and the seeded input generators); it is
run by hand, in parallel over seeds:
    python tests/golden/make_longrun_profiles.py [--procs 8]
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N0 = 40_000
WARM = 4
MEASURE = 20
SEEDS = list(range(1, 9))
OUT = os.path.join(HERE, "longrun_c1_profiles.json")


def case_for(seed):
    from paper_2103_09642_amd.workloads import base_case
    return base_case(n_init_e=N0, n_init_i=N0, weight=3.5e5 * 1000 / N0, seed=seed,
                     flags=["density", "meane"])


def run(seed):
    from oracle import binding as orc
    from paper_2103_09642_amd.workloads import synthetic_xsec
    c = case_for(seed)
    o = orc.Oracle(c, synthetic_xsec())
    o.seed()
    t0 = time.time()
    o.step(WARM * c["steps_per_cycle"])
    o.reset_diag()
    o.step(MEASURE * c["steps_per_cycle"])
    ne, ni = o.density()
    me = o.mean_energy()
    return {"seed": seed, "ne": ne.tolist(), "ni": ni.tolist(), "mean_energy": me.tolist(),
            "n_e": o.count(0), "n_i": o.count(1), "counts": o.counts(), "seconds": time.time() - t0}


def rel_l2(a, b, mask):
    return float(np.linalg.norm(a[mask] - b[mask]) / np.linalg.norm(b[mask]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    args = ap.parse_args()
    with Pool(args.procs) as p:
        res = p.map(run, SEEDS)
    mean = {key: np.mean([r[key] for r in res], axis=0) for key in ("ne", "ni", "mean_energy")}
    mask = mean["ne"] >= 0.1 * mean["ne"].max()
    spread = {}
    for key in ("ne", "ni", "mean_energy"):
        spread[key] = [rel_l2(np.asarray(r[key]), mean[key], mask) for r in res]
    def sig(v):  # six significant digits keep the file small
        return [float("%.6g" % x) for x in v]
    out = {"case": {"n0": N0, "weight": 3.5e5 * 1000 / N0, "warm_cycles": WARM, "measure_cycles": MEASURE,
                    "seeds": SEEDS, "geometry": "small plain case (400 nodes, 4000 steps/cycle, 10 Pa, 250 V)"},
           "generated_by": "tests/golden/make_longrun_profiles.py (oracle only)",
           "mean": {k: sig(v) for k, v in mean.items()},
           "spread_about_mean": {k: sig(v) for k, v in spread.items()},
           "seed_1": {k: sig(res[0][k]) for k in ("ne", "ni", "mean_energy")},
           "final_counts": [{"seed": r["seed"], "n_e": r["n_e"], "n_i": r["n_i"], "counts": r["counts"]}
                            for r in res]}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    for key, v in spread.items():
        print(key, "relative L2 about the mean: max %.4f mean %.4f" % (max(v), float(np.mean(v))))
    print("final counts", [(r["seed"], r["n_e"], r["n_i"], round(r["seconds"])) for r in res])


if __name__ == "__main__":
    main()
