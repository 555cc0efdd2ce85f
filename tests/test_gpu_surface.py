"""Surface processes on the GPU against the CPU oracle: elastic electron
reflection (eta_e) and ion-induced secondary emission (gamma) per electrode.

Bar as for the plain step: counters and deposits bit-exact, particle state
(matched by uid) within 1e-12 relative after one step; the secondaries'
velocities come from device log/cos/sin (libm ulps)."""
import numpy as np
import pytest

from gpu_common import compare_states, gpu_context, make_pair, say, set_both
from paper_2103_09642_amd.workloads import base_case, random_state

pytestmark = pytest.mark.gpu

QE, MAR = 1.602176634e-19, 39.948 * 1.66053906660e-27
COUNTERS = ("abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i", "ioniz", "see_pow", "see_gnd",
            "refl")


@pytest.fixture(scope="module")
def ctx(xs_default):
    c = gpu_context()
    c.set_xsec(xs_default)
    return c


def _case(**kw):
    kw.setdefault("n_init_e", 0)
    kw.setdefault("n_init_i", 0)
    kw.setdefault("flags", ["allow_unstable"])
    kw.setdefault("cap_e", 200_000)
    kw.setdefault("cap_i", 200_000)
    kw.setdefault("gamma_see", (0.3, 0.2))
    kw.setdefault("eta_refl", (0.4, 0.6))
    kw.setdefault("see_te_ev", 2.0)
    return base_case(**kw)


def _with_wall_particles(c, st, n, seed):
    """Add n electrons and n ions per electrode that leave the gap in the
    first push (ions: on an ion step)."""
    rng = np.random.default_rng(seed)
    L = c["gap_m"]
    out = {}
    for key, speed, reach in (("e", 3e6, 2e-5), ("i", np.sqrt(2 * 40 * QE / MAR), 1e-6)):
        d = rng.uniform(1e-9, reach, 2 * n)
        x = np.concatenate([d[:n], L - d[n:]])
        vx = np.concatenate([np.full(n, -speed), np.full(n, speed)])
        uid = rng.integers(1 << 50, 1 << 60, 2 * n, dtype=np.uint64)
        add = {"x": x, "vx": vx, "vy": rng.normal(0, speed / 10, 2 * n), "vz": rng.normal(0, speed / 10, 2 * n),
               "uid": uid}
        out[key] = {k: np.concatenate([st[key][k], add[k]]) for k in add}
    return out


@pytest.mark.parametrize("step", [0, 5])
def test_surface_one_step_parity(ctx, xs_default, orc, step):
    """One step with both processes at both electrodes: the same particles
    (reflected electrons kept, secondaries added with their identities),
    the same counters and deposits."""
    from paper_2103_09642_amd import edupic
    say(f"test_surface_one_step_parity step={step}")
    ctx.set_option(edupic.OPT_POISSON, edupic.POISSON_THOMAS)
    try:
        c = _case(pressure_pa=40.0, weight=2e5, ion_subcycle=5)
        st = random_state(40_000, 40_000, c["gap_m"], seed=31 + step, te_ev=4.0, hot_frac=0.3, hot_ev=80.0,
                          ion_energy_ev=40.0)
        st = _with_wall_particles(c, st, 2000, seed=step)
        g, o = make_pair(ctx, c, xs_default, orc)
        set_both(g, o, st, step)
        g.advance_steps(1)
        o.step(1)
        cg, co = g.counts(), o.counts()
        for k in COUNTERS:
            assert cg[k] == co[k], k
        assert co["refl"] > 500
        if step == 0:
            assert co["see_pow"] > 300 and co["see_gnd"] > 200
        for sp in (0, 1):
            compare_states(g.get_state(sp), o.get_state(sp), 1e-12, f"sp{sp}")
        ge, gi = g.deposit()
        oe, oi = o.deposit()
        assert np.array_equal(ge, oe) and np.array_equal(gi, oi)
        g.destroy()
    finally:
        ctx.set_option(edupic.OPT_POISSON, edupic.POISSON_FLUX)


@pytest.mark.parametrize("mode", [0, 1], ids=["plain", "graph"])
def test_surface_multi_step_parity(ctx, xs_default, orc, mode):
    """30 steps (6 ion steps) in plain and graph execution: counters equal
    and the particles equal to 1e-9 relative (collided particles carry
    libm-vs-device ulps)."""
    from paper_2103_09642_amd import edupic
    say(f"test_surface_multi_step_parity mode={mode}")
    ctx.set_option(edupic.OPT_POISSON, edupic.POISSON_THOMAS)
    ctx.set_option(edupic.OPT_MODE, mode)
    try:
        c = _case(pressure_pa=20.0, weight=2e5, ion_subcycle=5, gamma_see=(0.5, 0.5), eta_refl=(0.3, 0.3))
        st = random_state(30_000, 30_000, c["gap_m"], seed=41, te_ev=3.0, hot_frac=0.1, hot_ev=60.0,
                          ion_energy_ev=60.0)
        st = _with_wall_particles(c, st, 1000, seed=9)
        g, o = make_pair(ctx, c, xs_default, orc)
        set_both(g, o, st, 0)
        g.advance_steps(30)
        o.step(30)
        cg, co = g.counts(), o.counts()
        for k in COUNTERS:
            assert cg[k] == co[k], k
        assert co["see_pow"] > 0 and co["see_gnd"] > 0 and co["refl"] > 0
        for sp in (0, 1):
            compare_states(g.get_state(sp), o.get_state(sp), 1e-9, f"sp{sp}")
        g.destroy()
    finally:
        ctx.set_option(edupic.OPT_MODE, 0)
        ctx.set_option(edupic.OPT_POISSON, edupic.POISSON_FLUX)


def test_surface_parameters_are_validated(ctx):
    from paper_2103_09642_amd import edupic
    say("test_surface_parameters_are_validated")
    for bad in ({"gamma_see": (1.5, 0.0)}, {"eta_refl": (0.0, -0.1)}, {"see_te_ev": 0.0}):
        with pytest.raises(edupic.EdpError):
            ctx.case_bytes(_case(**bad))
