"""Long-run statistical parity with the oracle (section 3.5's time-averaged
density and mean-energy profiles).

PIC/MCC is chaotic: after a few thousand steps the GPU and oracle
trajectories separate through rounding differences (device vs libm ulps of
exp/log/sin/cos, the flux-form field solve), and any independent realisation
is an equally valid result.  Long runs are therefore compared on
time-averaged profiles, against the mean of eight oracle seeds stored in
tests/golden/longrun_c1_profiles.json by tests/golden/make_longrun_profiles.py
(a script that runs only the oracle).

The case is the small plain case's geometry and gas (2.5 cm, 10 Pa, 400
nodes, 4000 steps per 13.56 MHz period, 250 V), seeded with 4e4 + 4e4
particles; 4 RF cycles let the sheaths form, then 20 RF cycles are averaged.
The discharge is still growing then (it converges only over about 1500
cycles, beyond a test's budget), which is the same for both sides: they run
the same window from the same seeded state.

Bound: the relative L2 distance over the nodes where the mean n_e is at
least 10% of its maximum is at most 3% for n_e, n_i and the mean electron
energy.  The oracle's own seeds lie at most 1.2% (n_e), 1.4% (n_i) and 0.6%
(mean energy) from their mean (stored with the profiles and checked below),
so a GPU realisation from the same distribution passes with a margin of two,
while a systematic error of the size the bound names fails."""
import json
import os

import numpy as np
import pytest

from gpu_common import gpu_context, say
from paper_2103_09642_amd.workloads import base_case

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "longrun_c1_profiles.json")
BOUND = 0.03


def _rel_l2(a, b, mask):
    return float(np.linalg.norm(a[mask] - b[mask]) / np.linalg.norm(b[mask]))


@pytest.mark.parametrize("seed", [1, 2])
def test_time_averaged_profiles_match_the_oracle(xs_default, seed):
    with open(GOLDEN) as f:
        gold = json.load(f)
    cfg = gold["case"]
    mean = {k: np.asarray(v) for k, v in gold["mean"].items()}
    mask = mean["ne"] >= 0.1 * mean["ne"].max()
    # the test's power: the oracle's seed-to-seed scatter is well inside the bound
    for k, v in gold["spread_about_mean"].items():
        assert max(v) < BOUND / 2, (k, max(v))
    say(f"test_time_averaged_profiles_match_the_oracle seed={seed}: {int(mask.sum())} nodes")
    ctx = gpu_context()
    ctx.set_xsec(xs_default)
    c = base_case(n_init_e=cfg["n0"], n_init_i=cfg["n0"], weight=cfg["weight"], seed=seed,
                  flags=["density", "meane"])
    g = ctx.create_case(c)
    g.advance(cfg["warm_cycles"])
    g.reset_diag()
    g.advance(cfg["measure_cycles"])
    ne, ni = g.density()
    me = g.mean_energy()
    k = g.counts()
    got = {"ne": ne, "ni": ni, "mean_energy": me}
    dist = {key: _rel_l2(got[key], mean[key], mask) for key in got}
    say(f"  relative L2 vs the oracle mean: {dist}; live {k['n_e']} e, {k['n_i']} i; "
        f"oracle seed scatter {[max(v) for v in gold['spread_about_mean'].values()]}")
    g.destroy()
    ctx.close()
    for key, d in dist.items():
        assert d <= BOUND, f"{key}: relative L2 {d:.4f} > {BOUND}"
