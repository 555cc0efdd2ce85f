"""Seeded synthetic inputs: cross-section tables, case parameters, particle states.

This module holds no step of the PIC/MCC method itself.  It produces the
*inputs* the method takes -- cross-section tables, discharge parameters and
particle snapshots -- so that the GPU library and the CPU oracle can be fed
the same numbers.  Both sides convert a case dict into their own descriptor.

The paper's electron and Ar+ cross sections (Phelps, section 3.2) are not
available here, so the tables are smooth argon-like stand-ins with the
paper's structure: elastic, one lumped excitation (threshold 11.5 eV) and
ionization (15.8 eV) for electrons versus LAB energy; isotropic plus backward
elastic parts for Ar+ versus COM energy.  Tabulation follows section 3.2:
bin i <-> energy i * DE_CS, DE_CS = 1 meV.
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

# Constants used only to draw seed velocities and choose time steps.
_QE = 1.602176634e-19
_ME = 9.1093837015e-31
_KB = 1.380649e-23
_MAR = 39.948 * 1.66053906660e-27

CS_RANGES = 100_000
DE_CS = 1.0e-3
E_EXC_THR = 11.5
E_ION_THR = 15.8
W_IONIZ = 10.0
RF_FREQ = 13.56e6


def synthetic_xsec(n_bins: int = CS_RANGES, de_ev: float = DE_CS, scale: float = 1.0) -> Dict:
    """Argon-like tables [m^2].  Thresholds act on whole bins: a process is
    zero in every bin at or below round(threshold/de), so no bin sits partly
    above a threshold.  `scale` multiplies every cross section (used to force
    collisions in tests)."""
    i = np.arange(n_bins, dtype=np.float64)
    eps = i * de_ev
    el = 1e-20 + 2.8e-19 * (eps / 12.0) / (1.0 + (eps / 12.0) ** 2)
    exc = np.zeros(n_bins)
    ion = np.zeros(n_bins)
    k_exc = int(round(E_EXC_THR / de_ev))
    k_ion = int(round(E_ION_THR / de_ev))
    m = i > k_exc
    exc[m] = 5e-20 * np.log(eps[m] / E_EXC_THR) / (eps[m] / E_EXC_THR)
    m = i > k_ion
    ion[m] = 8e-20 * np.log(eps[m] / E_ION_THR) / (eps[m] / E_ION_THR)
    iso = 2e-19 / np.sqrt(eps + 0.01)
    back = 1e-19 / np.sqrt(eps + 0.01)
    return {
        "n_bins": n_bins, "de_ev": de_ev,
        "e_el": el * scale, "e_exc": exc * scale, "e_ion": ion * scale,
        "i_iso": iso * scale, "i_back": back * scale,
        "e_exc_thr_ev": E_EXC_THR, "e_ion_thr_ev": E_ION_THR, "w_ioniz_ev": W_IONIZ,
    }


def zero_xsec(n_bins: int = 1000, de_ev: float = DE_CS) -> Dict:
    """Collisionless tables (all cross sections zero)."""
    z = np.zeros(n_bins)
    return {"n_bins": n_bins, "de_ev": de_ev, "e_el": z, "e_exc": z, "e_ion": z,
            "i_iso": z, "i_back": z, "e_exc_thr_ev": E_EXC_THR,
            "e_ion_thr_ev": E_ION_THR, "w_ioniz_ev": W_IONIZ}


def base_case(**kw) -> Dict:
    """Reference-like defaults (Table 2 geometry and gas), overridable."""
    c = {
        "gap_m": 0.025, "pressure_pa": 10.0, "gas_temp_k": 350.0, "area_m2": 1e-4,
        "n_grid": 400, "steps_per_cycle": 4000, "ion_subcycle": 20,
        "dt_e": 1.0 / (RF_FREQ * 4000),
        "harmonics": [(250.0, RF_FREQ, 0.0)],
        "weight": 3.5e5, "n_init_e": 1000, "n_init_i": 1000,
        "te_init_ev": 2.0, "ti_init_k": 350.0, "seed": 1,
        "flags": [], "n_eepf": 2000, "de_eepf_ev": 0.05,
        # measurement mode: N_BIN steps per xt bin, IFEDF 200 x 1 eV (section 4.1)
        "n_xt_bin": 20, "n_ifed": 200, "de_ifed_ev": 1.0,
        # surface processes (section 5), (powered, grounded); off by default
        "gamma_see": (0.0, 0.0), "eta_refl": (0.0, 0.0), "see_te_ev": 1.0,
        "v_dc": 0.0,  # DC offset of the powered electrode (self-bias) [V]
    }
    c.update(kw)
    return c


def config_small() -> Dict:
    """Plain small case: 400 nodes, 4000 steps/period, 1000+1000 seeds,
    W = 3.5e5 (about 2e4 per species at the reference density), seed 1."""
    return base_case()


def config_large() -> Dict:
    """Plain large case: 1000 nodes, 8000 steps/period, a uniform plasma of
    1e15 m^-3 seeded as 2e6 electrons + 2e6 ions (W = 1250)."""
    n = 2_000_000
    return base_case(n_grid=1000, steps_per_cycle=8000, dt_e=1.0 / (RF_FREQ * 8000),
                     weight=1e15 * 1e-4 * 0.025 / n, n_init_e=n, n_init_i=n)


def _nu_max(pressure_pa: float, temp_k: float, xs: Dict) -> float:
    n = pressure_pa / (_KB * temp_k)
    eps = np.arange(xs["n_bins"]) * xs["de_ev"]
    v = np.sqrt(2.0 * eps * _QE / _ME)
    return float(np.max(n * (xs["e_el"] + xs["e_exc"] + xs["e_ion"]) * v))


def steps_per_cycle_rule(freq: float, dx: float, pressure_pa: float, temp_k: float,
                         xs: Dict) -> int:
    """Time steps per period that keep the collision probability below 0.05
    and a 30 eV electron under one cell per step (stability criteria 3-4),
    at least 2000, rounded up to a multiple of 20."""
    vstar = math.sqrt(2.0 * 30.0 * _QE / _ME)
    need = max(2000.0, vstar / (freq * dx), _nu_max(pressure_pa, temp_k, xs) / (freq * -math.log(0.95)))
    return int(20 * math.ceil(need / 20.0))


def config_batch(k: int, xs: Dict | None = None) -> Dict:
    """Batched-set case k (1..64): pressure log-uniform 5-100 Pa, voltage
    100-500 V, gap 1.5-5 cm, 200-1000 nodes, particle count log-uniform
    1e4-5e5 per species, 13.56 MHz, drawn with numpy.random.default_rng(k)."""
    xs = xs if xs is not None else synthetic_xsec()
    r = np.random.default_rng(k)
    p = math.exp(r.uniform(math.log(5.0), math.log(100.0)))
    v = r.uniform(100.0, 500.0)
    L = r.uniform(0.015, 0.05)
    ng = int(r.integers(200, 1001))
    n = int(math.exp(r.uniform(math.log(1e4), math.log(5e5))))
    nt = steps_per_cycle_rule(RF_FREQ, L / (ng - 1), p, 350.0, xs)
    return base_case(gap_m=L, pressure_pa=p, n_grid=ng, steps_per_cycle=nt,
                     dt_e=1.0 / (RF_FREQ * nt), harmonics=[(v, RF_FREQ, 0.0)],
                     weight=1e15 * 1e-4 * L / n, n_init_e=n, n_init_i=n, seed=k)


def config_dualfreq(k: int) -> Dict:
    """Dual-frequency case k (1..32): 2.5 cm, 2.5-20 Pa, V1 sin(2 pi 1.937 MHz t)
    + V2 sin(2 pi 27.12 MHz t); 2000 steps per 27.12 MHz period; 1000 nodes;
    1e6 per species.  One 'cycle' is one low-frequency period = 28002 steps."""
    r = np.random.default_rng(1000 + k)
    p = math.exp(r.uniform(math.log(2.5), math.log(20.0)))
    v1 = r.uniform(100.0, 400.0)
    v2 = r.uniform(50.0, 200.0)
    dt = 1.0 / (27.12e6 * 2000)
    spc = int(round((1.0 / 1.937e6) / dt))
    n = 1_000_000
    return base_case(pressure_pa=p, n_grid=1000, steps_per_cycle=spc, dt_e=dt,
                     harmonics=[(v1, 1.937e6, 0.0), (v2, 27.12e6, 0.0)],
                     weight=1e15 * 1e-4 * 0.025 / n, n_init_e=n, n_init_i=n, seed=k)


# ---------------------------------------------------------------------------
# Particle snapshots for parity tests
# ---------------------------------------------------------------------------

def maxwellian(rng: np.random.Generator, n: int, kt_j: float, mass: float) -> np.ndarray:
    return rng.normal(0.0, math.sqrt(kt_j / mass), size=(3, n))


def random_state(n_e: int, n_i: int, gap_m: float, seed: int, te_ev: float = 3.0,
                 ti_k: float = 350.0, hot_frac: float = 0.05, hot_ev: float = 60.0,
                 edge_cases: bool = True, ion_energy_ev: float = 0.0) -> Dict:
    """A snapshot with both species: uniform positions, Maxwellian velocities,
    plus a fraction of hot electrons (uniform 0..hot_ev eV, isotropic) so that
    excitation and ionization occur within a step.  With edge_cases the first
    particles sit exactly at x = 0, x = L, on a node, and just inside/outside
    the walls after one push.  uids are distinct 64-bit values."""
    rng = np.random.default_rng(seed)
    out = {}
    for sp, n in (("e", n_e), ("i", n_i)):
        x = rng.uniform(0.0, gap_m, size=n)
        if sp == "e":
            v = maxwellian(rng, n, te_ev * _QE, _ME)
            nh = int(hot_frac * n)
            if nh:
                en = rng.uniform(0.0, hot_ev, size=nh)
                sp_ = np.sqrt(2.0 * en * _QE / _ME)
                mu = rng.uniform(-1.0, 1.0, size=nh)
                ph = rng.uniform(0.0, 2 * math.pi, size=nh)
                st = np.sqrt(1.0 - mu * mu)
                v[0, :nh] = sp_ * mu
                v[1, :nh] = sp_ * st * np.cos(ph)
                v[2, :nh] = sp_ * st * np.sin(ph)
        else:
            v = maxwellian(rng, n, _KB * ti_k, _MAR)
            if ion_energy_ev > 0.0 and n:
                m = n // 4
                v[0, :m] += rng.choice([-1.0, 1.0], size=m) * math.sqrt(2 * ion_energy_ev * _QE / _MAR)
        if edge_cases and n >= 8:
            x[0] = 0.0
            x[1] = gap_m
            x[2] = gap_m / 2.0
            x[3] = 1e-12 * gap_m
            x[4] = gap_m * (1.0 - 1e-12)
            v[:, 0:2] = 0.0
            # heading out fast: absorbed after the push
            v[0, 3] = -3e6 if sp == "e" else -3e4
            v[0, 4] = 3e6 if sp == "e" else 3e4
        uid = rng.integers(0, 2**63 - 1, size=n, dtype=np.int64).astype(np.uint64)
        uid = np.unique(uid)
        while uid.size < n:  # practically never
            extra = rng.integers(0, 2**63 - 1, size=n - uid.size, dtype=np.int64).astype(np.uint64)
            uid = np.unique(np.concatenate([uid, extra]))
        rng.shuffle(uid)
        out[sp] = {"x": np.ascontiguousarray(x), "vx": np.ascontiguousarray(v[0]),
                   "vy": np.ascontiguousarray(v[1]), "vz": np.ascontiguousarray(v[2]),
                   "uid": np.ascontiguousarray(uid[:n])}
    return out


def serving_stream(rate_hz: float, duration_s: float, seed: int = 0, p_large: float = 0.1,
                   cyc_lo: int = 20, cyc_hi: int = 200) -> List[Dict]:
    """Poisson arrivals of requests; each is a large-type case with probability
    p_large, else a batched-set case, asking for a number of RF cycles drawn
    uniformly from cyc_lo..cyc_hi."""
    r = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += r.exponential(1.0 / rate_hz)
        if t > duration_s:
            break
        large = r.uniform() < p_large
        k = int(r.integers(1, 65))
        out.append({"t_arrival": t, "kind": "large" if large else "batch", "case_k": k,
                    "cycles": int(r.integers(cyc_lo, cyc_hi + 1))})
    return out
