"""The outer control loops (section 5: DC self-bias, power target) on model
plants whose response is known in closed form, and their actuator on the
oracle."""
import math

import numpy as np
import pytest

from paper_2103_09642_amd import control
from paper_2103_09642_amd.workloads import RF_FREQ, base_case, random_state


class PowerPlant:
    """P = a * V^2 (V the amplitude sum): the target is reached at
    V* = sqrt(P_t / a)."""

    def __init__(self, a):
        self.a, self.v = a, 0.0

    def set_voltage(self, v_amp, v_dc):
        self.v = float(np.sum(v_amp))

    def reset_diag(self):
        pass

    def info(self):
        return {"power_e": 0.3 * self.a * self.v ** 2, "power_i": 0.7 * self.a * self.v ** 2}


class BiasPlant:
    """Charges to the powered electrode per window: N (1 + t) / 2 positive
    and N (1 - t) / 2 negative with t = tanh((V_eq - V_dc) / s): balanced at
    V_dc = V_eq, more ions when the bias is below it."""

    def __init__(self, v_eq, s=30.0, n=10**6):
        self.v_eq, self.s, self.n = v_eq, s, n
        self.v_dc = 0.0
        self.c = {"abs_i_pow": 0, "see_pow": 0, "abs_e_pow": 0}

    def set_voltage(self, v_amp, v_dc):
        self.v_dc = v_dc

    def counts(self):
        return dict(self.c)

    def step(self):
        t = math.tanh((self.v_eq - self.v_dc) / self.s)
        pos = int(round(self.n * (1 + t) / 2))
        self.c["abs_i_pow"] += pos - pos // 10
        self.c["see_pow"] += pos // 10
        self.c["abs_e_pow"] += self.n - pos


def _advance_counter():
    calls = []

    def adv(plants, steps):
        calls.append((len(plants), steps))
        for p in plants:
            if hasattr(p, "step"):
                p.step()
    return adv, calls


def test_power_loop_converges_for_low_gain_in_one_batch():
    """Three plants in one loop (one advance per window for all of them)
    reach V* = sqrt(P_t/a) within the tolerance; with gain < 1/2 the
    approach from below is monotone."""
    plants = [PowerPlant(a) for a in (0.01, 0.04, 0.2)]
    cases = [base_case(harmonics=[(100.0, RF_FREQ, 0.0)]) for _ in plants]
    adv, calls = _advance_counter()
    res = control.power_target(plants, cases, adv, 400, target_w_m3=2000.0, gain=0.4, tol=1e-3)
    for p, lc in zip(plants, res):
        assert lc.converged
        vstar = math.sqrt(2000.0 / p.a)
        assert float(lc.v_amp.sum()) == pytest.approx(vstar, rel=2e-3)
        v = [float(h["v_amp"].sum()) for h in lc.history]
        if v[0] < vstar:
            assert all(b >= a for a, b in zip(v, v[1:]))
    assert calls[0] == (3, 400) and all(n <= 3 for n, _ in calls)
    assert len(calls) == max(len(lc.history) for lc in res)


def test_power_loop_with_high_gain_does_not_settle():
    """gain 1.2: the error is multiplied by about |1 - 2 gain| = 1.4 per
    window, so the loop oscillates instead of converging."""
    p = PowerPlant(0.04)
    adv, _ = _advance_counter()
    res = control.power_target([p], [base_case(harmonics=[(180.0, RF_FREQ, 0.0)])], adv, 10,
                               target_w_m3=2000.0, gain=1.2, tol=1e-3, max_iter=40)
    assert not res[0].converged
    err = [h["power"] / 2000.0 - 1 for h in res[0].history]
    assert any(e > 0 for e in err) and any(e < 0 for e in err)


def test_power_loop_clamps_each_step():
    p = PowerPlant(1e-6)  # far too little power: every window asks for the most
    adv, _ = _advance_counter()
    res = control.power_target([p], [base_case(harmonics=[(100.0, RF_FREQ, 0.0)])], adv, 10,
                               target_w_m3=2000.0, gain=0.3, clamp=1.25, max_iter=5)
    v = [float(h["v_amp"].sum()) for h in res[0].history]
    assert np.allclose(np.array(v[1:]) / np.array(v[:-1]), 1.25)


def test_self_bias_finds_the_balance_point():
    """The bias settles where the electrode's charges balance, for an
    equilibrium below and above the start."""
    plants = [BiasPlant(-85.0), BiasPlant(40.0)]
    cases = [base_case(harmonics=[(200.0, RF_FREQ, 0.0)]) for _ in plants]
    adv, calls = _advance_counter()
    res = control.self_bias(plants, cases, adv, 4000, gain=0.2, tol=0.005)
    for p, lc in zip(plants, res):
        assert lc.converged
        assert lc.v_dc == pytest.approx(p.v_eq, abs=0.5)
        assert abs(lc.history[-1]["imbalance"]) < 0.005
    assert calls[0] == (2, 4000)


def test_voltage_actuator_on_the_oracle(orc, xs_default):
    """set_voltage takes effect from the next step: phi at the powered
    electrode is the new waveform plus the DC offset, and a power loop on a
    small discharge moves the amplitude in the direction of the target."""
    c = base_case(steps_per_cycle=400, dt_e=1.0 / (RF_FREQ * 400), n_xt_bin=10, ion_subcycle=5,
                  pressure_pa=20.0, weight=1e6, n_init_e=0, n_init_i=0, flags=["xt", "density", "meane"],
                  harmonics=[(150.0, RF_FREQ, 0.0)])
    st = random_state(4000, 4000, c["gap_m"], seed=3, te_ev=3.0)
    o = orc.Oracle(c, xs_default)
    o.set_state(0, st["e"], 0)
    o.set_state(1, st["i"], 0)
    o.step(3)
    o.set_voltage([90.0], -12.5)
    o.step(1)
    _, phi, _ = o.fields()
    want = 90.0 * math.sin(2 * math.pi * RF_FREQ * 3 * c["dt_e"]) - 12.5
    assert phi[0] == pytest.approx(want, rel=1e-15, abs=1e-12)
    with pytest.raises(ValueError):
        o.set_voltage([1.0, 2.0], 0.0)
    # the loop asks for more power than 150 V gives: the amplitude rises
    res = control.power_target([o], [c], lambda ps, n: [p.step(n) for p in ps], 200,
                               target_w_m3=1e9, gain=0.3, max_iter=2)
    v = [float(h["v_amp"][0]) for h in res[0].history]
    assert v == [150.0, 150.0 * 1.25]
