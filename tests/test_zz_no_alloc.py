"""The allocation-free advance (edp_advance_steps_noalloc) against the
ordinary advance (edp_advance_steps), through the C ABI: the same cases
advanced both ways give bit-identical particles, deposits and counters, on
two calls in a row, the second with a smaller input (fewer, smaller cases,
fewer steps)."""
import numpy as np
import pytest

from gpu_common import by_uid, gpu_context, say
from paper_2103_09642_amd.workloads import base_case

pytestmark = pytest.mark.gpu


def _descs(sizes, seed0):
    return [base_case(n_init_e=n, n_init_i=n, weight=3e9 / n, pressure_pa=20.0 + 10 * k,
                      seed=seed0 + k, cap_e=4 * n, cap_i=4 * n, flags=["allow_unstable"])
            for k, n in enumerate(sizes)]


def _same(a, b, label):
    ca, cb = a.counts(), b.counts()
    assert ca == cb, (label, ca, cb)
    da, db = a.deposit(), b.deposit()
    assert np.array_equal(da[0], db[0]) and np.array_equal(da[1], db[1]), label
    for sp in (0, 1):
        sa, sb = by_uid(a.get_state(sp)), by_uid(b.get_state(sp))
        for k in ("uid", "x", "vx", "vy", "vz"):
            assert np.array_equal(sa[k], sb[k]), (label, sp, k)
    return ca


@pytest.mark.parametrize("calls", [[((60_000, 25_000, 9_000), 400), ((7_000,), 130)]])
def test_noalloc_advance_equals_the_ordinary_advance(xs_default, calls):
    ctx = gpu_context()
    ctx.set_xsec(xs_default)
    seed0 = 1
    for j, (sizes, steps) in enumerate(calls):
        say(f"test_noalloc call {j}: {len(sizes)} cases {sizes}, {steps} steps")
        ref = [ctx.create_case(d) for d in _descs(sizes, seed0)]
        new = [ctx.create_case(d) for d in _descs(sizes, seed0)]
        ctx.advance_steps(ref, [steps] * len(ref))
        ctx.advance_steps_noalloc(new, [steps] * len(new))
        ctx.sync()
        for k, (a, b) in enumerate(zip(ref, new)):
            c = _same(a, b, f"call {j} case {k}")
            assert c["step"] == steps and c["coll_e"] > 0 and c["n_e"] > 0
        for g in ref + new:
            g.destroy()
        seed0 += 10
    ctx.close()
