"""GPU path against the CPU oracle, through the C ABI.

Bar: integer work (deposits, counters, identities) bit-exact; FP64 particle
state within 1e-12 relative after one step from an identical state (the push
is bit-identical by construction; collided particles differ only through
libm-vs-device ulps of exp/log/sin/cos/tan/atan)."""
import math

import numpy as np
import pytest

from gpu_common import by_uid, compare_states, gpu_context, make_pair, poisson_reference, say, set_both
from paper_2103_09642_amd.workloads import base_case, random_state, synthetic_xsec, zero_xsec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(xs_default):
    c = gpu_context()
    c.set_xsec(xs_default)
    return c


def _case(**kw):
    kw.setdefault("n_init_e", 0)
    kw.setdefault("n_init_i", 0)
    kw.setdefault("flags", ["allow_unstable"])
    return base_case(**kw)


def test_seed_matches_oracle(ctx, xs_default, orc):
    """Seeding draws from Philox: positions x = L u are bit-exact, so the
    device Philox equals the oracle's; velocities agree to libm ulps."""
    say("test_seed_matches_oracle")
    c = base_case(n_init_e=50_000, n_init_i=30_000, weight=1.0)
    g, o = make_pair(ctx, c, xs_default, orc)
    o.seed()
    for sp in (0, 1):
        a, b = by_uid(g.get_state(sp)), by_uid(o.get_state(sp))
        assert np.array_equal(a["uid"], b["uid"])
        assert np.array_equal(a["x"], b["x"])
        compare_states(a, b, 1e-13, f"seed sp{sp}")
    ge, gi = g.deposit()
    oe, oi = o.deposit()
    assert np.array_equal(ge, oe) and np.array_equal(gi, oi)
    g.destroy()


@pytest.mark.parametrize("ng,nsub,n", [(400, 20, 30_000), (17, 3, 5_000), (1000, 1, 60_000), (2, 5, 2_000)])
def test_deposit_bit_exact(ctx, xs_default, orc, ng, nsub, n):
    """Fixed-point densities of an identical state are bit-identical,
    including particles on nodes, at x = 0 and x = L."""
    say(f"test_deposit_bit_exact ng={ng} nsub={nsub} n={n}")
    c = _case(n_grid=ng, ion_subcycle=nsub, cap_e=n + 4096, cap_i=n + 4096)
    g, o = make_pair(ctx, c, xs_default, orc)
    st = random_state(n, n // 2, c["gap_m"], seed=ng + n)
    for step in (0, 7):
        set_both(g, o, st, step)
        ge, gi = g.deposit()
        oe, oi = o.deposit()
        assert np.array_equal(ge, oe)
        assert np.array_equal(gi, oi)
        assert ge.sum() == n * 2**32 and gi.sum() == (n // 2) * 2**32
    g.destroy()


def _one_step(ctx, xs, orc, c, st, step, nsteps=1):
    g, o = make_pair(ctx, c, xs, orc)
    set_both(g, o, st, step)
    g.advance_steps(nsteps)
    o.step(nsteps)
    return g, o


@pytest.fixture
def poisson(ctx, request):
    from paper_2103_09642_amd import edupic
    ctx.set_option(edupic.OPT_POISSON, request.param)
    yield request.param
    ctx.set_option(edupic.OPT_POISSON, edupic.POISSON_FLUX)


@pytest.mark.parametrize("pretest", [0, 2], ids=["auto", "by-energy"])
@pytest.mark.parametrize("poisson", [1, 0], indirect=True, ids=["thomas", "flux"])
@pytest.mark.parametrize("step", [0, 5])
def test_one_step_parity(ctx, xs_default, orc, step, poisson, pretest):
    """One full step (ion step and electron-only step) from an identical
    state with hot electrons, high pressure (many collisions incl.
    ionization) and particles at/near both walls.  With the sequential
    Thomas solve the fields are bit-identical; with the parallel flux solve
    they agree to 1e-12 of the field scale, and the deposit after the step is
    compared with the oracle's deposit of the GPU's own positions.  The
    collision pre-test runs with its automatic bound (here P* over the whole
    table) and with the bound by energy block forced."""
    from paper_2103_09642_amd import edupic
    say(f"test_one_step_parity step={step} poisson={poisson} pretest={pretest}")
    ctx.set_option(edupic.OPT_PRETEST, pretest)
    c = _case(pressure_pa=50.0, weight=2e5, n_grid=400, ion_subcycle=5, cap_e=200_000, cap_i=200_000)
    st = random_state(60_000, 50_000, c["gap_m"], seed=11 + step, te_ev=4.0, hot_frac=0.3, hot_ev=90.0,
                      ion_energy_ev=30.0)
    g, o = _one_step(ctx, xs_default, orc, c, st, step)
    rg, pg, eg = g.fields()
    ro, po, eo = o.fields()
    assert np.array_equal(rg, ro), "rho"
    if poisson == 1:
        assert np.array_equal(pg, po), "phi (Thomas, same operation order)"
        assert np.array_equal(eg, eo), "E"
    else:
        # the flux solve is within 1e-14 of an 80-bit solution; the oracle's
        # sequential Thomas sweep carries ~1e-13 rounding of its own
        dx = c["gap_m"] / (c["n_grid"] - 1)
        v_left = float(pg[0])
        eref = poisson_reference(rg, dx, v_left)
        assert float(np.max(np.abs(eg - eref))) <= 1e-14 * float(np.abs(eref).max()), "E vs extended precision"
        assert np.max(np.abs(eg - eo)) <= 1e-12 * np.abs(eo).max(), "E"
        assert np.max(np.abs(pg - po)) <= 1e-12 * np.abs(po).max(), "phi"
    cg, co = g.counts(), o.counts()
    for k in ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz", "anomaly"):
        assert cg[k if k != "anomaly" else "anomalies"] == co[k], k
    assert co["coll_e"] > 100 and co["ioniz"] > 10 and co["abs_e_pow"] + co["abs_e_gnd"] > 0
    if step % 5 == 0:
        assert co["coll_i"] > 10
    m = 0
    # a field difference dE moves v_x by dE*factor: judge v_x on the scale of
    # one step's largest field kick as well
    kick = {0: np.abs(eo).max() * c["dt_e"] * 1.602176634e-19 / 9.1093837015e-31,
            1: np.abs(eo).max() * c["dt_e"] * c["ion_subcycle"] * 1.602176634e-19 / (39.948 * 1.66053906660e-27)}
    for sp in (0, 1):
        fl = {k: kick[sp] for k in ("vx", "vy", "vz")}  # collisions mix the components
        m += compare_states(g.get_state(sp), o.get_state(sp), 1e-12, f"sp{sp}", floors=fl if poisson == 0 else None)
    ge, gi = g.deposit()
    oe, oi = o.deposit()
    if poisson == 1:
        assert np.array_equal(ge, oe), "electron deposit after the step"
        assert np.array_equal(gi, oi), "ion deposit after the step"
    else:
        inv_dx = 1.0 / (c["gap_m"] / (c["n_grid"] - 1))
        assert np.array_equal(ge, orc.deposit(g.get_state(0)["x"], c["n_grid"], inv_dx))
        assert int(ge.sum()) == int(oe.sum())  # same electrons
        # ions: the density held until the next ion step
        assert np.array_equal(gi, oi)
    say(f"  bit mismatches in state components: {m}")
    g.destroy()
    ctx.set_option(edupic.OPT_PRETEST, 0)


def test_multi_step_parity_and_subcycling(ctx, xs_default, orc):
    """60 steps (4 ion steps at N_SUB = 20) with births and absorption: the
    particle sets stay identical and the states agree to 1e-9."""
    say("test_multi_step_parity_and_subcycling")
    c = _case(pressure_pa=20.0, weight=1e5, n_grid=300, cap_e=100_000, cap_i=100_000)
    st = random_state(20_000, 20_000, c["gap_m"], seed=3, te_ev=3.0, hot_frac=0.2, hot_ev=80.0)
    g, o = _one_step(ctx, xs_default, orc, c, st, 0, nsteps=60)
    cg, co = g.counts(), o.counts()
    for k in ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz"):
        assert cg[k] == co[k], k
    for sp in (0, 1):
        compare_states(g.get_state(sp), o.get_state(sp), 1e-9, f"sp{sp}")
    g.destroy()


def test_empty_case_gives_vacuum_field(ctx, orc):
    """No particles: rho = 0 and E = V(t)/L on every node."""
    say("test_empty_case_gives_vacuum_field")
    xs = zero_xsec(n_bins=100_000)
    c = _case(harmonics=[(100.0, 0.0, math.pi / 2)])
    g, o = make_pair(ctx, c, xs, orc)
    empty = {k: np.zeros(0) for k in ("x", "vx", "vy", "vz")} | {"uid": np.zeros(0, np.uint64)}
    set_both(g, o, {"e": empty, "i": empty}, 0)
    g.advance_steps(3)
    o.step(3)
    _, pg, eg = g.fields()
    _, po, eo = o.fields()
    assert np.allclose(eg, eo, rtol=1e-13)
    assert np.allclose(pg, po, rtol=0, atol=1e-12 * 100.0)
    assert np.allclose(eg, 100.0 / c["gap_m"], rtol=1e-10)
    assert g.counts()["n_e"] == 0
    g.destroy()


def test_run_twice_and_launch_shape_are_bit_identical(ctx, xs_default):
    """Same state several times, with different compaction/sort intervals
    (different particle orders and chunk assignments) and with hipGraph
    capture: bit-identical particles, deposits and counters (integer
    deposits, counter-based random numbers keyed by particle identity)."""
    say("test_run_twice_and_launch_shape_are_bit_identical")
    from paper_2103_09642_amd import edupic
    c = _case(pressure_pa=30.0, weight=1e5, cap_e=120_000, cap_i=120_000)
    st = random_state(40_000, 40_000, c["gap_m"], seed=9, te_ev=3.0, hot_frac=0.2, hot_ev=70.0)
    res = []
    for mode, sort_every in ((0, 100), (0, 7), (1, 5), (0, 1000), (1, 1)):
        ctx.set_option(edupic.OPT_MODE, mode)
        ctx.set_option(edupic.OPT_SORT_EVERY, sort_every)
        g = ctx.create_case(c)
        g.set_state(0, st["e"], 0)
        g.set_state(1, st["i"], 0)
        g.advance_steps(200)
        res.append((by_uid(g.get_state(0)), by_uid(g.get_state(1)), g.deposit(), g.counts()))
        g.destroy()
    ctx.set_option(edupic.OPT_MODE, 0)
    ctx.set_option(edupic.OPT_SORT_EVERY, 100)
    for r in res[1:]:
        for sp in (0, 1):
            for k in ("uid", "x", "vx", "vy", "vz"):
                assert np.array_equal(res[0][sp][k], r[sp][k]), k
        assert np.array_equal(res[0][2][0], r[2][0]) and np.array_equal(res[0][2][1], r[2][1])
        assert res[0][3] == r[3]


def test_capacity_overflow_is_reported(ctx, xs_default):
    """Births beyond the capacity are dropped, counted, and edp_sync returns
    EDP_ECAPACITY; the case then refuses to advance."""
    say("test_capacity_overflow_is_reported")
    from paper_2103_09642_amd import edupic
    c = _case(pressure_pa=80.0, weight=1e5, cap_e=4096, cap_i=4096)
    st = random_state(4000, 4000, c["gap_m"], seed=1, te_ev=5.0, hot_frac=0.9, hot_ev=99.0)
    g = ctx.create_case(c)
    g.set_state(0, st["e"], 0)
    g.set_state(1, st["i"], 0)
    g.advance_steps(50)
    with pytest.raises(edupic.EdpError) as ei:
        ctx.sync()
    assert ei.value.code == edupic.EDP_ECAPACITY
    assert g.counts()["dropped"] > 0
    with pytest.raises(edupic.EdpError):
        g.advance_steps(1)
    g.destroy()


def test_invalid_descriptors_rejected(ctx):
    say("test_invalid_descriptors_rejected")
    from paper_2103_09642_amd import edupic
    for bad in (dict(n_grid=1), dict(n_grid=5000), dict(ion_subcycle=0), dict(dt_e=0.0),
                dict(harmonics=[(1.0, 1.0, 0.0)] * 5)):
        with pytest.raises((edupic.EdpError, ValueError)):
            ctx.create_case(_case(**bad))
    # stability check (omega_pe dt >= 2 at the seed density)
    with pytest.raises(edupic.EdpError) as ei:
        ctx.create_case(base_case(n_init_e=1000, n_init_i=1000, weight=1e13))
    assert ei.value.code == edupic.EDP_EUNSTABLE


@pytest.mark.parametrize("meane", [True, False], ids=["all", "no-meane"])
def test_diagnostics_match_oracle(ctx, xs_default, orc, meane):
    """Density, EEPF, currents and mean energy after 40 steps with every
    measurement on: density and EEPF counts bit-exact (integer deposits of
    identical positions), currents and mean energy to 1e-12.  Without the
    mean energy the streaming loop reads v_y and v_z only for the EEPF's
    window."""
    say(f"test_diagnostics_match_oracle meane={meane}")
    c = _case(pressure_pa=10.0, weight=1e5,
              flags=["allow_unstable", "density", "eepf", "current"] + (["meane"] if meane else []),
              cap_e=100_000, cap_i=100_000)
    st = random_state(30_000, 30_000, c["gap_m"], seed=4, te_ev=3.0, hot_frac=0.05, hot_ev=30.0)
    g, o = _one_step(ctx, xs_default, orc, c, st, 0, nsteps=40)
    ng_, ni_ = g.density()
    no_, nio = o.density()
    assert np.allclose(ng_, no_, rtol=1e-10, atol=1e-10 * no_.max())
    assert np.allclose(ni_, nio, rtol=1e-10, atol=1e-10 * nio.max())
    fg, cg = g.eepf()
    fo, co = o.eepf()
    assert cg.sum() == co.sum() and np.abs(cg - co).max() <= 2
    jg = g.currents()
    jo = o.currents()
    for a, b in zip(jg, jo):
        assert np.allclose(a, b, rtol=1e-9, atol=1e-9 * np.abs(b).max())
    if meane:
        mg, mo = g.mean_energy(), o.mean_energy()
        assert np.allclose(mg, mo, rtol=1e-9, atol=1e-9 * mo.max())
    g.destroy()


# ---------------------------------------------------------------------------
# Full size: the benchmark's case (1000 nodes, 8000 steps per period,
# 2e6 + 2e6 seeded particles, W = 1250) in the benchmark's launch setup.
# ---------------------------------------------------------------------------

def test_full_size_two_steps_match_oracle(ctx, xs_default, orc):
    """Both sides seed the benchmark case from Philox and run two steps (an
    ion step, then an electron-only step); every one of the ~4e6 particles is
    compared by uid, plus counters, rho and the deposit of the GPU's own
    positions."""
    say("test_full_size_two_steps_match_oracle")
    from paper_2103_09642_amd import workloads
    c = workloads.config_large()
    g = ctx.create_case(c)
    o = orc.Oracle(c, xs_default)
    o.seed()
    g.advance_steps(2)
    o.step(2)
    cg, co = g.counts(), o.counts()
    for k in ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz"):
        assert cg[k] == co[k], k
    assert co["coll_e"] > 1000 and co["coll_i"] > 100
    rg, _, eg = g.fields()
    ro, _, eo = o.fields()
    assert np.array_equal(rg, ro), "rho"
    assert np.max(np.abs(eg - eo)) <= 1e-12 * np.abs(eo).max(), "E"
    kick = {0: np.abs(eo).max() * c["dt_e"] * 1.602176634e-19 / 9.1093837015e-31,
            1: np.abs(eo).max() * c["dt_e"] * c["ion_subcycle"] * 1.602176634e-19 / (39.948 * 1.66053906660e-27)}
    for sp in (0, 1):
        a, b = g.get_state(sp), o.get_state(sp)
        assert a["uid"].size == cg["n_e" if sp == 0 else "n_i"]
        compare_states(a, b, 1e-12, f"full sp{sp}", floors={k: kick[sp] for k in ("vx", "vy", "vz")})
    ge, _ = g.deposit()
    inv_dx = 1.0 / (c["gap_m"] / (c["n_grid"] - 1))
    assert np.array_equal(ge, orc.deposit(g.get_state(0)["x"], c["n_grid"], inv_dx))
    g.destroy()


def test_full_size_graph_run_matches_plain_and_keeps_invariants(ctx, xs_default):
    """2000 steps of the benchmark case captured as hipGraphs (the timed
    configuration) give bit-identical particles, deposits and counters to
    plain launches, and the run keeps the bookkeeping invariants: live
    counts = seeded - absorbed + births, deposit sum = 2^32 per live
    particle, every particle inside [0, L] with finite velocity."""
    say("test_full_size_graph_run_matches_plain_and_keeps_invariants")
    from paper_2103_09642_amd import edupic, workloads
    c = workloads.config_large()
    res = []
    for mode in (1, 0):
        ctx.set_option(edupic.OPT_MODE, mode)
        g = ctx.create_case(c)
        g.advance_steps(2000)
        res.append((by_uid(g.get_state(0)), by_uid(g.get_state(1)), g.deposit(), g.counts()))
        g.destroy()
    ctx.set_option(edupic.OPT_MODE, 0)
    (e1, i1, d1, k1), (e0, i0, d0, k0) = res
    assert k1 == k0
    for a, b in ((e1, e0), (i1, i0)):
        for k in ("uid", "x", "vx", "vy", "vz"):
            assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(d1[0], d0[0]) and np.array_equal(d1[1], d0[1])
    n0 = c["n_init_e"]
    assert k1["n_e"] == n0 - k1["abs_e_pow"] - k1["abs_e_gnd"] + k1["ioniz"] - k1["dropped"]
    assert k1["n_i"] == n0 - k1["abs_i_pow"] - k1["abs_i_gnd"] + k1["ioniz"] - k1["dropped"]
    assert k1["dropped"] == 0 and k1["step"] == 2000
    assert e1["uid"].size == k1["n_e"] and i1["uid"].size == k1["n_i"]
    assert int(d1[0].sum()) == k1["n_e"] * 2**32
    for st_ in (e1, i1):
        assert np.all((st_["x"] >= 0.0) & (st_["x"] <= c["gap_m"]))
        for k in ("vx", "vy", "vz"):
            assert np.all(np.isfinite(st_[k]))
    assert np.unique(e1["uid"]).size == e1["uid"].size and np.unique(i1["uid"]).size == i1["uid"].size


# Long runs are compared statistically, on time-averaged profiles over 20 RF
# cycles against eight oracle seeds: tests/test_gpu_longrun.py.


# ---------------------------------------------------------------------------
# Null-collision selection (section 2.1.6): same random slots as the direct
# test, so the GPU and the oracle make the same decisions.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("step", [0, 5])
def test_null_collision_one_step_parity(ctx, xs_default, orc, step):
    say(f"test_null_collision_one_step_parity step={step}")
    c = _case(pressure_pa=50.0, weight=2e5, n_grid=400, ion_subcycle=5, cap_e=200_000, cap_i=200_000,
              flags=["allow_unstable", "null_collision"])
    st = random_state(60_000, 50_000, c["gap_m"], seed=31 + step, te_ev=4.0, hot_frac=0.3, hot_ev=90.0,
                      ion_energy_ev=30.0)
    g, o = _one_step(ctx, xs_default, orc, c, st, step)
    cg, co = g.counts(), o.counts()
    for k in ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz", "anomaly"):
        assert cg[k if k != "anomaly" else "anomalies"] == co[k], k
    assert co["coll_e"] > 100 and co["ioniz"] > 10
    if step % 5 == 0:
        assert co["coll_i"] > 10
    _, _, eo = o.fields()
    kick = {0: np.abs(eo).max() * c["dt_e"] * 1.602176634e-19 / 9.1093837015e-31,
            1: np.abs(eo).max() * c["dt_e"] * c["ion_subcycle"] * 1.602176634e-19 / (39.948 * 1.66053906660e-27)}
    for sp in (0, 1):
        compare_states(g.get_state(sp), o.get_state(sp), 1e-12, f"null sp{sp}",
                       floors={k: kick[sp] for k in ("vx", "vy", "vz")})
    g.destroy()


def test_null_collision_multi_step_parity(ctx, xs_default, orc):
    say("test_null_collision_multi_step_parity")
    c = _case(pressure_pa=20.0, weight=1e5, n_grid=300, cap_e=100_000, cap_i=100_000,
              flags=["allow_unstable", "null_collision"])
    st = random_state(20_000, 20_000, c["gap_m"], seed=33, te_ev=3.0, hot_frac=0.2, hot_ev=80.0)
    g, o = _one_step(ctx, xs_default, orc, c, st, 0, nsteps=60)
    cg, co = g.counts(), o.counts()
    for k in ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz"):
        assert cg[k] == co[k], k
    for sp in (0, 1):
        compare_states(g.get_state(sp), o.get_state(sp), 1e-9, f"null sp{sp}")
    g.destroy()


def _thomas(ctx):
    from paper_2103_09642_amd import edupic
    ctx.set_option(edupic.OPT_POISSON, edupic.POISSON_THOMAS)


def _flux(ctx):
    from paper_2103_09642_amd import edupic
    ctx.set_option(edupic.OPT_POISSON, edupic.POISSON_FLUX)


@pytest.mark.parametrize("step", [0, 5])
def test_every_particle_a_candidate_flushes_segments(ctx, xs_default, orc, step):
    """Cross sections x30 (ions x1200) at 30 Pa make nearly every particle a
    collision candidate, and 1.5e6 particles per species give every particle workgroup several
    chunks: each wave's candidate segment fills and is processed inside the
    loop, the rest at the workgroup's end.  One step (ion step and
    electron-only step) against the oracle: counters exact, particles to
    1e-12, deposits exact (Thomas solve)."""
    say(f"test_every_particle_a_candidate_flushes_segments step={step}")
    xs = synthetic_xsec(scale=30.0)
    xs["i_iso"], xs["i_back"] = xs["i_iso"] * 40.0, xs["i_back"] * 40.0
    ctx.set_xsec(xs)
    _thomas(ctx)
    try:
        n = 1_500_000
        c = _case(pressure_pa=30.0, weight=3e4, ion_subcycle=5, cap_e=2 * n, cap_i=2 * n)
        st = random_state(n, n, c["gap_m"], seed=61 + step, te_ev=3.0, hot_frac=0.05, hot_ev=40.0,
                          ion_energy_ev=20.0)
        g, o = make_pair(ctx, c, xs, orc)
        set_both(g, o, st, step)
        g.advance_steps(1)
        o.step(1)
        cg, co = g.counts(), o.counts()
        for k in ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz", "anomaly"):
            assert cg[k if k != "anomaly" else "anomalies"] == co[k], k
        assert co["coll_e"] > n // 10
        if step == 0:
            assert co["coll_i"] > n // 20
        for sp in (0, 1):
            compare_states(g.get_state(sp), o.get_state(sp), 1e-12, f"sp{sp}")
        ge, gi = g.deposit()
        oe, oi = o.deposit()
        assert np.array_equal(ge, oe) and np.array_equal(gi, oi)
        g.destroy()
    finally:
        ctx.set_xsec(xs_default)
        _flux(ctx)


def test_energetic_particles_beyond_the_bound_range(ctx, xs_default, orc):
    """Electrons of 0.5-3 keV and ions of 1-3 keV lie beyond the energy range
    the collision-probability bound covers (four times the table range), so
    they are tested exactly whatever their uniform: one ion step against the
    oracle, counters exact, particles to 1e-12."""
    say("test_energetic_particles_beyond_the_bound_range")
    _thomas(ctx)
    try:
        c = _case(pressure_pa=50.0, weight=2e5, ion_subcycle=5, cap_e=200_000, cap_i=200_000)
        st = random_state(40_000, 40_000, c["gap_m"], seed=71, te_ev=3.0)
        rng = np.random.default_rng(72)
        for key, mass, lo, hi in (("e", 9.1093837015e-31, 500.0, 3000.0),
                                  ("i", 39.948 * 1.66053906660e-27, 1000.0, 3000.0)):
            m = 8000
            en = rng.uniform(lo, hi, m)
            d = rng.normal(size=(3, m))
            d /= np.linalg.norm(d, axis=0)
            sp_ = np.sqrt(2 * en * 1.602176634e-19 / mass)
            for k, comp in zip(("vx", "vy", "vz"), d):
                st[key][k][-m:] = sp_ * comp
        g, o = make_pair(ctx, c, xs_default, orc)
        set_both(g, o, st, 0)
        g.advance_steps(1)
        o.step(1)
        cg, co = g.counts(), o.counts()
        for k in ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz", "anomaly"):
            assert cg[k if k != "anomaly" else "anomalies"] == co[k], k
        assert co["ioniz"] > 100 and co["coll_i"] > 10
        for sp in (0, 1):
            compare_states(g.get_state(sp), o.get_state(sp), 1e-12, f"sp{sp}")
        g.destroy()
    finally:
        _flux(ctx)
