"""The persistent small-case kernel (EDP_OPT_SMALL_MAX): one workgroup
advances one case through a window of steps in one launch.  It is the same
method as the lockstep path, so the same cases give bit-identical particles,
deposits and counters either way -- alone, in a batch with cases on the
lockstep path, and when a case switches between the two paths -- and it
matches the oracle like the lockstep path does."""
import numpy as np
import pytest

from gpu_common import by_uid, compare_states, gpu_context, make_pair, say, set_both
from paper_2103_09642_amd.workloads import base_case, random_state

pytestmark = pytest.mark.gpu

KEYS = ("uid", "x", "vx", "vy", "vz")


@pytest.fixture(scope="module")
def ctx(xs_default):
    c = gpu_context()
    c.set_xsec(xs_default)
    return c


@pytest.fixture
def small(ctx):
    from paper_2103_09642_amd import edupic

    def set_(v):
        ctx.set_option(edupic.OPT_SMALL_MAX, v)
    yield set_
    set_(0)
    ctx.set_option(edupic.OPT_POISSON, edupic.POISSON_FLUX)
    ctx.set_option(edupic.OPT_SORT_EVERY, 100)


def _snap(g):
    return (by_uid(g.get_state(0)), by_uid(g.get_state(1)), g.deposit(), g.counts())


def _same(a, b, label):
    assert a[3] == b[3], (label, a[3], b[3])
    for sp in (0, 1):
        for k in KEYS:
            assert np.array_equal(a[sp][k], b[sp][k]), (label, sp, k)
    assert np.array_equal(a[2][0], b[2][0]) and np.array_equal(a[2][1], b[2][1]), label


def _hot_case(**kw):
    kw.setdefault("flags", ["allow_unstable"])
    return base_case(n_init_e=0, n_init_i=0, pressure_pa=40.0, weight=1e6, ion_subcycle=5,
                     cap_e=40_000, cap_i=40_000, **kw)


def _state(c, seed, n=6000):
    return random_state(n, n, c["gap_m"], seed=seed, te_ev=4.0, hot_frac=0.3, hot_ev=90.0, ion_energy_ev=40.0)


@pytest.mark.parametrize("flags", [["allow_unstable"],
                                   ["allow_unstable", "density", "eepf", "current", "meane", "xt", "ifed"],
                                   ["allow_unstable", "null_collision"]],
                         ids=["plain", "measure", "null"])
def test_small_equals_lockstep(ctx, small, flags):
    """300 steps (sorts every 7 steps, ion steps every 5, reflection and
    secondary emission on) give the same bits in the small-case kernel as on
    the lockstep path, measurements included."""
    from paper_2103_09642_amd import edupic
    say(f"test_small_equals_lockstep {flags}")
    ctx.set_option(edupic.OPT_SORT_EVERY, 7)
    c = _hot_case(flags=flags, gamma_see=(0.2, 0.1), eta_refl=(0.2, 0.3), see_te_ev=2.0, n_grid=300)
    st = _state(c, 81)
    res = []
    # the small-case kernel with the pre-test's bound by energy block forced
    for lim, pre in ((0, 0), (10**9, 2)):
        small(lim)
        ctx.set_option(edupic.OPT_PRETEST, pre)
        g = ctx.create_case(c)
        g.set_state(0, st["e"], 0)
        g.set_state(1, st["i"], 0)
        g.advance_steps(300)
        snap = _snap(g)
        extra = ()
        if "density" in flags:
            extra = (g.density(), g.eepf()[1], g.currents(), g.mean_energy(), g.xt("ne"), g.ifed()[2])
        res.append((snap, extra))
        g.destroy()
    ctx.set_option(edupic.OPT_PRETEST, 0)
    _same(res[0][0], res[1][0], "small vs lockstep")
    assert res[0][0][3]["coll_e"] > 1000 and res[0][0][3]["ioniz"] > 10
    for a, b in zip(res[0][1], res[1][1]):
        for x, y in zip(a if isinstance(a, tuple) else (a,), b if isinstance(b, tuple) else (b,)):
            assert np.array_equal(x, y)


def test_switching_paths_and_mixed_batch(ctx, small):
    """A case that switches lockstep -> small -> lockstep (the slot counts
    and birth counters handed over at each switch) ends where a
    lockstep-only run ends, and a batch
    mixing small cases (on their own stream) with a large lockstep case
    gives every case the bits it gets alone."""
    say("test_switching_paths_and_mixed_batch")
    c = _hot_case()
    st = _state(c, 82)
    small(0)
    ref = ctx.create_case(c)
    ref.set_state(0, st["e"], 0)
    ref.set_state(1, st["i"], 0)
    ref.advance_steps(240)
    want = _snap(ref)
    ref.destroy()
    g = ctx.create_case(c)
    g.set_state(0, st["e"], 0)
    g.set_state(1, st["i"], 0)
    g.advance_steps(77)
    small(10**9)
    g.advance_steps(90)
    small(0)
    g.advance_steps(73)
    _same(want, _snap(g), "switching")
    g.destroy()
    # mixed batch: two small cases and one large case (above the limit)
    big = base_case(n_init_e=0, n_init_i=0, pressure_pa=20.0, weight=1e5, cap_e=200_000, cap_i=200_000,
                    flags=["allow_unstable"])
    sb = random_state(60_000, 60_000, big["gap_m"], seed=83)
    descs = [(c, _state(c, 84)), (dict(c, n_grid=150), _state(c, 85, 3000)), (big, sb)]
    alone = []
    for d, s in descs:
        small(20_000)
        g = ctx.create_case(d)
        g.set_state(0, s["e"], 0)
        g.set_state(1, s["i"], 0)
        g.advance_steps(130)
        alone.append(_snap(g))
        g.destroy()
    small(20_000)
    gs = []
    for d, s in descs:
        g = ctx.create_case(d)
        g.set_state(0, s["e"], 0)
        g.set_state(1, s["i"], 0)
        gs.append(g)
    ctx.advance_steps(gs, [130, 130, 130])
    for k, g in enumerate(gs):
        _same(alone[k], _snap(g), f"mixed case {k}")
        g.destroy()


def test_small_matches_oracle(ctx, xs_default, orc, small):
    """With the sequential Thomas solve, 60 steps in the small-case kernel
    follow the oracle: counters exactly, particles within 1e-9."""
    from paper_2103_09642_amd import edupic
    say("test_small_matches_oracle")
    small(10**9)
    ctx.set_option(edupic.OPT_POISSON, edupic.POISSON_THOMAS)
    c = _hot_case(gamma_see=(0.2, 0.1), eta_refl=(0.2, 0.3), see_te_ev=2.0)
    st = _state(c, 86)
    g, o = make_pair(ctx, c, xs_default, orc)
    set_both(g, o, st, 0)
    g.advance_steps(60)
    o.step(60)
    cg, co = g.counts(), o.counts()
    for k in ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz",
              "see_pow", "see_gnd", "refl"):
        assert cg[k] == co[k], k
    assert cg["n_e"] == o.count(0) and cg["n_i"] == o.count(1)
    for sp in (0, 1):
        compare_states(g.get_state(sp), o.get_state(sp), 1e-9, f"sp{sp}")
    g.destroy()
