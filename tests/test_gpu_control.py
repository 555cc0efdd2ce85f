"""Outer control loops (section 5) on the GPU: the waveform actuator against
the oracle, and the power and self-bias loops run side by side on library
cases (batched windows) and on oracle cases."""
import math

import numpy as np
import pytest

from gpu_common import compare_states, gpu_context, make_pair, say, set_both
from paper_2103_09642_amd import control
from paper_2103_09642_amd.workloads import RF_FREQ, base_case, random_state, zero_xsec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(xs_default):
    from paper_2103_09642_amd import edupic
    c = gpu_context()
    c.set_xsec(xs_default)
    c.set_option(edupic.OPT_POISSON, edupic.POISSON_THOMAS)
    yield c
    c.set_option(edupic.OPT_POISSON, edupic.POISSON_FLUX)


def _case(**kw):
    kw.setdefault("n_init_e", 0)
    kw.setdefault("n_init_i", 0)
    kw.setdefault("cap_e", 100_000)
    kw.setdefault("cap_i", 100_000)
    kw.setdefault("harmonics", [(150.0, RF_FREQ, 0.0)])
    return base_case(steps_per_cycle=400, dt_e=1.0 / (RF_FREQ * 400), n_xt_bin=10, ion_subcycle=5,
                     pressure_pa=20.0, weight=1e6, **kw)


def test_set_voltage_parity(ctx, xs_default, orc):
    """A new amplitude and DC offset between advances: the next steps see
    the same waveform on both sides (fields bit-identical with Thomas)."""
    say("test_set_voltage_parity")
    c = _case(flags=["allow_unstable"])
    st = random_state(20_000, 20_000, c["gap_m"], seed=2, te_ev=3.0)
    g, o = make_pair(ctx, c, xs_default, orc)
    set_both(g, o, st, 0)
    g.advance_steps(3)
    o.step(3)
    for p in (g, o):
        p.set_voltage([90.0], -12.5)
    g.advance_steps(2)
    o.step(2)
    rg, pg, eg = g.fields()
    ro, po, eo = o.fields()
    assert np.array_equal(pg, po) and np.array_equal(eg, eo)
    assert pg[0] == pytest.approx(90.0 * math.sin(2 * math.pi * RF_FREQ * 4 * c["dt_e"]) - 12.5, abs=1e-12)
    for sp in (0, 1):
        compare_states(g.get_state(sp), o.get_state(sp), 1e-12, f"sp{sp}")
    from paper_2103_09642_amd import edupic
    with pytest.raises(edupic.EdpError):
        g.set_voltage([1.0, 2.0], 0.0)
    g.destroy()


def _oracle_advance(plants, steps):
    for p in plants:
        p.step(steps)


def _collisionless_pair(ctx, xs_default, orc, c, st):
    """A library case and an oracle case without collisions: with the
    Thomas solve their steps stay bit-identical over many windows (with
    collisions, an ulp of exp can flip a collision test now and then and
    the runs drift apart by single particles)."""
    xs0 = zero_xsec()
    ctx.set_xsec(xs0)
    try:
        g, o = make_pair(ctx, c, xs0, orc)
    finally:
        ctx.set_xsec(xs_default)
    set_both(g, o, st, 0)
    return g, o


def test_power_loop_matches_oracle(ctx, xs_default, orc):
    """Three windows of the power loop on two collisionless library cases
    (one batched advance per window) and on the same cases in the oracle:
    the same measured powers and amplitudes, to 1e-9."""
    say("test_power_loop_matches_oracle")
    cases = [_case(flags=["allow_unstable", "xt"], seed=s, harmonics=[(v, RF_FREQ, 0.0)])
             for s, v in ((1, 150.0), (2, 220.0))]
    gs, os_ = [], []
    for k, c in enumerate(cases):
        st = random_state(15_000, 15_000, c["gap_m"], seed=10 + k, te_ev=3.0, hot_frac=0.1, hot_ev=50.0)
        g, o = _collisionless_pair(ctx, xs_default, orc, c, st)
        gs.append(g)
        os_.append(o)
    kw = dict(window_steps=100, target_w_m3=5e4, gain=0.3, max_iter=3)
    rg = control.power_target(gs, cases, control.gpu_advance(ctx), **kw)
    ro = control.power_target(os_, cases, _oracle_advance, **kw)
    for a, b in zip(rg, ro):
        assert len(a.history) == len(b.history) == 3
        msg = f"gpu {[(h['power'], h['v_amp'][0]) for h in a.history]} oracle {[(h['power'], h['v_amp'][0]) for h in b.history]}"
        say(msg)
        for ha, hb in zip(a.history, b.history):
            assert ha["power"] == pytest.approx(hb["power"], rel=1e-9), msg
            assert np.allclose(ha["v_amp"], hb["v_amp"], rtol=1e-9), msg
    for g in gs:
        g.destroy()


def test_self_bias_loop_matches_oracle(ctx, xs_default, orc):
    """Three windows of the self-bias loop with unequal secondary yields on
    a collisionless case: the same electrode charges and DC offsets as the
    oracle."""
    say("test_self_bias_loop_matches_oracle")
    c = _case(flags=["allow_unstable"], gamma_see=(0.4, 0.0), see_te_ev=2.0)
    st = random_state(20_000, 20_000, c["gap_m"], seed=5, te_ev=3.0, ion_energy_ev=40.0)
    g, o = _collisionless_pair(ctx, xs_default, orc, c, st)
    kw = dict(window_steps=100, gain=0.2, tol=1e-9, max_iter=3)
    rg = control.self_bias([g], [c], control.gpu_advance(ctx), **kw)
    ro = control.self_bias([o], [c], _oracle_advance, **kw)
    msg = f"gpu {rg[0].history} oracle {ro[0].history}"
    say(msg)
    for ha, hb in zip(rg[0].history, ro[0].history):
        assert ha["charges"] == hb["charges"], msg
        assert ha["v_dc"] == pytest.approx(hb["v_dc"], rel=1e-12, abs=1e-12)
    assert rg[0].history[-1]["charges"] > 0
    g.destroy()
