"""Whole-step pins for the oracle: bookkeeping, determinism, diagnostics."""
import math

import numpy as np
import pytest

from paper_2103_09642_amd.workloads import base_case, random_state, synthetic_xsec, zero_xsec

QE, ME = 1.602176634e-19, 9.1093837015e-31


def _sorted(st):
    o = np.argsort(st["uid"])
    return {k: v[o] for k, v in st.items()}


def _empty():
    return {k: np.zeros(0) for k in ("x", "vx", "vy", "vz")} | {"uid": np.zeros(0, np.uint64)}


@pytest.fixture(scope="module")
def hot_case(xs_default):
    # dense, hot, high pressure: absorption and ionization every step
    c = base_case(pressure_pa=60.0, weight=2e5, n_init_e=0, n_init_i=0, ion_subcycle=4)
    st = random_state(20_000, 20_000, c["gap_m"], seed=5, te_ev=4.0, hot_frac=0.3, hot_ev=90.0)
    return c, st


def test_particle_bookkeeping_per_step(orc, xs_default, hot_case):
    """N_e(s+1) = N_e(s) - absorbed_e + births, N_i likewise on every step,
    and every ionization makes one electron and one ion."""
    c, st = hot_case
    o = orc.Oracle(c, xs_default)
    o.set_state(0, st["e"], 0)
    o.set_state(1, st["i"], 0)
    prev = o.counts()
    ne, ni = st["e"]["x"].size, st["i"]["x"].size
    for _ in range(12):
        o.step(1)
        cur = o.counts()
        d = {k: cur[k] - prev[k] for k in cur}
        ne2 = o.get_state(0)["x"].size
        ni2 = o.get_state(1)["x"].size
        assert ne2 == ne - d["abs_e_pow"] - d["abs_e_gnd"] + d["ioniz"]
        assert ni2 == ni - d["abs_i_pow"] - d["abs_i_gnd"] + d["ioniz"]
        ne, ni, prev = ne2, ni2, cur
    assert cur["ioniz"] > 0 and cur["abs_e_pow"] + cur["abs_e_gnd"] > 0 and cur["coll_i"] > 0
    assert cur["anomaly"] == 0
    uids = o.get_state(0)["uid"]
    assert np.unique(uids).size == uids.size


def test_result_independent_of_particle_order(orc, xs_default, hot_case):
    """Counter-based random numbers keyed by particle identity and integer
    deposits make the step independent of storage order: a permuted input
    gives the same particles (sorted by uid) bit for bit."""
    c, st = hot_case
    rng = np.random.default_rng(0)
    res = []
    for perm in (False, True):
        o = orc.Oracle(c, xs_default)
        for sp, key in ((0, "e"), (1, "i")):
            s = st[key]
            if perm:
                p = rng.permutation(s["x"].size)
                s = {k: v[p] for k, v in s.items()}
            o.set_state(sp, s, 0)
        o.step(9)
        res.append((_sorted(o.get_state(0)), _sorted(o.get_state(1)), o.counts(), o.deposit()))
    for k in ("x", "vx", "vy", "vz", "uid"):
        assert np.array_equal(res[0][0][k], res[1][0][k])
        assert np.array_equal(res[0][1][k], res[1][1][k])
    assert res[0][2] == res[1][2]
    assert np.array_equal(res[0][3][0], res[1][3][0])


def test_density_normalisation(orc):
    """A static neutral plasma: the time average equals the instantaneous
    density, and the grid integral with half cells at the edges gives W N / A
    (edge doubling of Algorithm 2)."""
    c = base_case(harmonics=[], weight=5e4, n_init_e=0, n_init_i=0, flags=["density"])
    o = orc.Oracle(c, zero_xsec())
    rng = np.random.default_rng(3)
    n = 5000
    x = rng.uniform(0, c["gap_m"], n)
    x[:2] = [0.0, c["gap_m"]]
    st = {"x": x, "vx": np.zeros(n), "vy": np.zeros(n), "vz": np.zeros(n), "uid": np.arange(n, dtype=np.uint64)}
    o.set_state(0, st, 0)
    o.set_state(1, st, 0)
    o.step(3)
    ne, ni = o.density()
    assert np.array_equal(ne, ni)
    dx = c["gap_m"] / (c["n_grid"] - 1)
    w = np.full(c["n_grid"], dx)
    w[0] = w[-1] = dx / 2
    assert (ne * w).sum() == pytest.approx(c["weight"] * n / c["area_m2"], rel=1e-12)
    _, _, E = o.fields()
    assert np.all(E == 0.0)


def test_current_and_mean_energy_diagnostics(orc):
    """Current density j = -e n vbar for a uniform drift, mean energy equals
    the common kinetic energy, EEPF integrates to one (sum f sqrt(eps) de = 1)."""
    c = base_case(harmonics=[], weight=5e4, n_init_e=0, n_init_i=0,
                  flags=["density", "current", "meane", "eepf"])
    o = orc.Oracle(c, zero_xsec())
    rng = np.random.default_rng(4)
    n = 20_000
    x = rng.uniform(0.3, 0.7, n) * c["gap_m"]
    vd = 1.0e3  # tiny drift: particles move far less than a cell in one step
    vy = 6.0e5
    e = {"x": x, "vx": np.full(n, vd), "vy": np.full(n, vy), "vz": np.zeros(n), "uid": np.arange(n, dtype=np.uint64)}
    i = {"x": x.copy(), "vx": np.zeros(n), "vy": np.zeros(n), "vz": np.zeros(n), "uid": np.arange(n, dtype=np.uint64)}
    o.set_state(0, e, 0)
    o.set_state(1, i, 0)
    o.step(1)
    ne, _ = o.density()
    je, ji = o.currents()
    m = ne > 0
    assert np.allclose(je[m], -QE * ne[m] * vd, rtol=1e-5)
    assert np.all(je[~m] == 0) and np.all(ji == 0)
    mee = o.mean_energy()
    en = 0.5 * ME * (vd * vd + vy * vy) / QE
    assert np.allclose(mee[m], en, rtol=1e-5)
    f, cnt = o.eepf()
    de = c["de_eepf_ev"]
    eps = (np.arange(c["n_eepf"]) + 0.5) * de
    assert (f * np.sqrt(eps) * de).sum() == pytest.approx(1.0, rel=1e-12)
    inside = np.sum((x >= 0.45 * c["gap_m"]) & (x <= 0.55 * c["gap_m"]))
    assert cnt.sum() == inside and cnt[int(en / de)] == inside


def test_eepf_of_a_maxwellian(orc):
    """A Maxwellian at k T = 2 eV (no field, no collisions): ln f is linear in
    eps with slope -1/kT (the EEPF of section 3.5)."""
    c = base_case(harmonics=[], weight=0.0, n_init_e=200_000, n_init_i=0, te_init_ev=2.0,
                  flags=["eepf"])
    o = orc.Oracle(c, zero_xsec())
    o.seed()
    o.step(1)
    f, cnt = o.eepf()
    de = c["de_eepf_ev"]
    eps = (np.arange(c["n_eepf"]) + 0.5) * de
    m = (eps > 0.5) & (eps < 8.0) & (cnt > 50)
    slope = np.polyfit(eps[m], np.log(f[m]), 1, w=np.sqrt(cnt[m]))[0]
    assert slope == pytest.approx(-1.0 / 2.0, rel=0.03)


def test_seeded_run_is_deterministic(orc, xs_default):
    """Same case, same seed: identical particles and counters."""
    c = base_case(n_init_e=3000, n_init_i=3000, weight=3e6)
    outs = []
    for _ in range(2):
        o = orc.Oracle(c, xs_default)
        o.seed()
        o.step(60)
        outs.append((_sorted(o.get_state(0)), o.counts()))
    assert outs[0][1] == outs[1][1]
    for k in ("x", "vx", "uid"):
        assert np.array_equal(outs[0][0][k], outs[1][0][k])


def test_voltage_waveform(orc):
    """V(t_s) with t_s = s dt_e; a cosine is the sine with phase pi/2."""
    c = base_case(harmonics=[(250.0, 13.56e6, math.pi / 2), (40.0, 27.12e6, 0.0)])
    o = orc.Oracle(c, zero_xsec())
    assert o.voltage(0) == pytest.approx(250.0, rel=1e-15)
    dt = c["dt_e"]
    for s in (1, 1000, 3999):
        t = s * dt
        want = 250 * math.cos(2 * math.pi * 13.56e6 * t) + 40 * math.sin(2 * math.pi * 27.12e6 * t)
        assert o.voltage(s) == pytest.approx(want, abs=1e-9)
    # one RF period later the single-frequency part repeats (N_t dt = T)
    c1 = base_case(harmonics=[(250.0, 13.56e6, 0.0)])
    o1 = orc.Oracle(c1, zero_xsec())
    assert o1.voltage(1234) == pytest.approx(o1.voltage(1234 + 4000), abs=1e-9)
