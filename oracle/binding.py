"""ctypes binding of the CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  It builds its own descriptor structs from a case dict; it does
not import the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

DIAG_DENSITY, DIAG_EEPF, DIAG_CURRENT, DIAG_MEANE, IONIZ_LITERAL = 1, 2, 4, 8, 16
NULL_COLLISION, DIAG_XT, DIAG_IFED = 64, 128, 256
_FLAG_NAMES = {"density": DIAG_DENSITY, "eepf": DIAG_EEPF, "current": DIAG_CURRENT,
               "meane": DIAG_MEANE, "ioniz_literal": IONIZ_LITERAL, "null_collision": NULL_COLLISION,
               "xt": DIAG_XT, "ifed": DIAG_IFED,
               "allow_unstable": 0}  # a library option with no effect on the method
XT_NAMES = ["pot", "efield", "ne", "ni", "je", "ji", "powere", "poweri", "meanee", "meanei", "ioniz"]
INFO_NAMES = ["mean_e", "ne_max", "debye", "dx_debye", "wpe_dt", "pmax_e", "pmax_i", "cfl_ev",
              "power_e", "power_i", "flux_i_pow", "flux_i_gnd", "ei_pow", "ei_gnd", "fail"]
COUNTER_NAMES = ["abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e", "coll_i",
                 "ioniz", "anomaly", "see_pow", "see_gnd", "refl"]


class OrcCase(C.Structure):
    _fields_ = [("gap_m", C.c_double), ("pressure_pa", C.c_double), ("gas_temp_k", C.c_double),
                ("area_m2", C.c_double), ("n_grid", C.c_int32), ("steps_per_cycle", C.c_int32),
                ("ion_subcycle", C.c_int32), ("n_harm", C.c_int32), ("dt_e", C.c_double),
                ("v_amp", C.c_double * 4), ("freq_hz", C.c_double * 4),
                ("phase_rad", C.c_double * 4), ("weight", C.c_double),
                ("n_init_e", C.c_int64), ("n_init_i", C.c_int64), ("te_init_ev", C.c_double),
                ("ti_init_k", C.c_double), ("seed", C.c_uint64), ("flags", C.c_uint32),
                ("n_eepf", C.c_int32), ("de_eepf_ev", C.c_double),
                ("n_xt_bin", C.c_int32), ("n_ifed", C.c_int32), ("de_ifed_ev", C.c_double),
                ("gamma_see", C.c_double * 2), ("eta_refl", C.c_double * 2), ("see_te_ev", C.c_double),
                ("v_dc", C.c_double)]


class OrcXsec(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("de_ev", C.c_double),
                ("e_el", C.POINTER(C.c_double)), ("e_exc", C.POINTER(C.c_double)),
                ("e_ion", C.POINTER(C.c_double)), ("i_iso", C.POINTER(C.c_double)),
                ("i_back", C.POINTER(C.c_double)), ("e_exc_thr_ev", C.c_double),
                ("e_ion_thr_ev", C.c_double), ("w_ioniz_ev", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int64)
        up = C.POINTER(C.c_uint64)
        L.orc_new.restype = P
        L.orc_new.argtypes = [C.POINTER(OrcCase), C.POINTER(OrcXsec)]
        L.orc_free.argtypes = [P]
        L.orc_error.restype = C.c_char_p
        L.orc_seed.argtypes = [P]
        L.orc_set_state.argtypes = [P, C.c_int, dp, dp, dp, dp, up, C.c_int64, C.c_int64]
        L.orc_get_state.restype = C.c_int64
        L.orc_get_state.argtypes = [P, C.c_int, dp, dp, dp, dp, up, C.c_int64]
        L.orc_step.argtypes = [P, C.c_int64]
        L.orc_count.restype = C.c_int64
        L.orc_count.argtypes = [P, C.c_int]
        L.orc_step_index.restype = C.c_int64
        L.orc_step_index.argtypes = [P]
        L.orc_counts.argtypes = [P, ip]
        L.orc_deposit_state.argtypes = [P, ip, ip]
        L.orc_fields.argtypes = [P, dp, dp, dp]
        L.orc_read_density.argtypes = [P, dp, dp]
        L.orc_read_eepf.argtypes = [P, dp, ip]
        L.orc_read_currents.argtypes = [P, dp, dp]
        L.orc_read_mean_energy.argtypes = [P, dp]
        L.orc_reset_diag.argtypes = [P]
        L.orc_n_xt.restype = C.c_int32
        L.orc_n_xt.argtypes = [P]
        L.orc_read_xt.argtypes = [P, C.c_int, dp]
        L.orc_xt_steps.argtypes = [P, ip, ip]
        L.orc_read_ifed.argtypes = [P, dp, dp, ip]
        L.orc_info.argtypes = [P, dp]
        L.orc_plasma_params.argtypes = [C.c_double, C.c_double, dp]
        L.orc_constants.argtypes = [P, dp]
        L.orc_voltage.restype = C.c_double
        L.orc_voltage.argtypes = [P, C.c_int64]
        L.orc_set_voltage.restype = C.c_int
        L.orc_set_voltage.argtypes = [P, dp, C.c_int32, C.c_double]
        L.orc_nsig_tot.argtypes = [P, dp, dp]
        L.orc_null_params.argtypes = [P, dp]
        L.orc_nu_star.restype = C.c_double
        L.orc_nu_star.argtypes = [dp, C.c_int32, C.c_double, C.c_double]
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                        C.POINTER(C.c_uint32)]
        L.orc_uniform2.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                   C.c_uint32, dp]
        L.orc_mix64.restype = C.c_uint64
        L.orc_mix64.argtypes = [C.c_uint64]
        L.orc_child_uid.restype = C.c_uint64
        L.orc_child_uid.argtypes = [C.c_uint64, C.c_int64, C.c_uint64]
        L.orc_deposit.argtypes = [dp, C.c_int64, C.c_int32, C.c_double, ip]
        L.orc_energy_bin.argtypes = [P, C.c_double]
        L.orc_energy_bin.restype = C.c_int
        L.orc_poisson.argtypes = [C.c_int32, C.c_double, dp, C.c_double, dp]
        L.orc_efield.argtypes = [C.c_int32, C.c_double, dp, dp, dp]
        L.orc_scatter.argtypes = [dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                  C.c_double, C.c_double, dp, dp]
        L.orc_collide_electron.restype = C.c_int
        L.orc_collide_electron.argtypes = [P, dp, C.c_int, C.c_double, C.c_double, C.c_double,
                                           C.c_double, dp, dp, C.POINTER(C.c_int)]
        L.orc_collide_ion.restype = C.c_int
        L.orc_collide_ion.argtypes = [P, dp, dp, C.c_int, C.c_double, C.c_double, C.c_double, dp]
        _lib = L
    return _lib


def dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def iptr(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def uptr(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def make_case(c: Dict) -> OrcCase:
    d = OrcCase()
    d.gap_m, d.pressure_pa, d.gas_temp_k, d.area_m2 = c["gap_m"], c["pressure_pa"], c["gas_temp_k"], c["area_m2"]
    d.n_grid, d.steps_per_cycle, d.ion_subcycle = c["n_grid"], c["steps_per_cycle"], c["ion_subcycle"]
    h = c["harmonics"]
    d.n_harm = len(h)
    for k, (v, f, ph) in enumerate(h):
        d.v_amp[k], d.freq_hz[k], d.phase_rad[k] = v, f, ph
    d.dt_e, d.weight = c["dt_e"], c["weight"]
    d.n_init_e, d.n_init_i = c["n_init_e"], c["n_init_i"]
    d.te_init_ev, d.ti_init_k, d.seed = c["te_init_ev"], c["ti_init_k"], c["seed"]
    fl = 0
    for name in c.get("flags", []):
        fl |= _FLAG_NAMES[name]
    d.flags = fl
    d.n_eepf, d.de_eepf_ev = c["n_eepf"], c["de_eepf_ev"]
    d.n_xt_bin = c.get("n_xt_bin", 20)
    d.n_ifed, d.de_ifed_ev = c.get("n_ifed", 200), c.get("de_ifed_ev", 1.0)
    d.gamma_see[0], d.gamma_see[1] = c.get("gamma_see", (0.0, 0.0))
    d.eta_refl[0], d.eta_refl[1] = c.get("eta_refl", (0.0, 0.0))
    d.see_te_ev = c.get("see_te_ev", 1.0)
    d.v_dc = c.get("v_dc", 0.0)
    return d


class Oracle:
    """One oracle case; the tables are copied in."""

    def __init__(self, case: Dict, xs: Dict):
        L = lib()
        self.case = case
        self.ng = case["n_grid"]
        self._arrs = [np.ascontiguousarray(xs[k], dtype=np.float64)
                      for k in ("e_el", "e_exc", "e_ion", "i_iso", "i_back")]
        x = OrcXsec()
        x.n_bins, x.de_ev = xs["n_bins"], xs["de_ev"]
        x.e_el, x.e_exc, x.e_ion, x.i_iso, x.i_back = (dptr(a) for a in self._arrs)
        x.e_exc_thr_ev, x.e_ion_thr_ev, x.w_ioniz_ev = xs["e_exc_thr_ev"], xs["e_ion_thr_ev"], xs["w_ioniz_ev"]
        self._desc = make_case(case)
        self.h = L.orc_new(C.byref(self._desc), C.byref(x))
        if not self.h:
            raise ValueError("oracle: " + L.orc_error().decode())

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def seed(self):
        lib().orc_seed(self.h)

    def set_state(self, species: int, st: Dict, step: int):
        a = {k: np.ascontiguousarray(st[k], dtype=np.float64) for k in ("x", "vx", "vy", "vz")}
        u = np.ascontiguousarray(st["uid"], dtype=np.uint64)
        n = a["x"].size
        lib().orc_set_state(self.h, species, dptr(a["x"]), dptr(a["vx"]), dptr(a["vy"]),
                            dptr(a["vz"]), uptr(u), n, step)

    def get_state(self, species: int) -> Dict:
        L = lib()
        n = L.orc_get_state(self.h, species, None, None, None, None, None, 0)
        out = {k: np.empty(n) for k in ("x", "vx", "vy", "vz")}
        out["uid"] = np.empty(n, dtype=np.uint64)
        L.orc_get_state(self.h, species, dptr(out["x"]), dptr(out["vx"]), dptr(out["vy"]),
                        dptr(out["vz"]), uptr(out["uid"]), n)
        return out

    def step(self, n: int = 1):
        lib().orc_step(self.h, n)

    def count(self, species: int) -> int:
        return lib().orc_count(self.h, species)

    @property
    def step_index(self) -> int:
        return lib().orc_step_index(self.h)

    def counts(self) -> Dict[str, int]:
        a = np.zeros(len(COUNTER_NAMES), dtype=np.int64)
        lib().orc_counts(self.h, iptr(a))
        return dict(zip(COUNTER_NAMES, (int(v) for v in a)))

    def deposit(self):
        ce = np.zeros(self.ng, dtype=np.int64)
        ci = np.zeros(self.ng, dtype=np.int64)
        lib().orc_deposit_state(self.h, iptr(ce), iptr(ci))
        return ce, ci

    def fields(self):
        rho, phi, E = (np.zeros(self.ng) for _ in range(3))
        lib().orc_fields(self.h, dptr(rho), dptr(phi), dptr(E))
        return rho, phi, E

    def density(self):
        ne, ni = np.zeros(self.ng), np.zeros(self.ng)
        lib().orc_read_density(self.h, dptr(ne), dptr(ni))
        return ne, ni

    def eepf(self):
        n = self.case["n_eepf"]
        f = np.zeros(n)
        c = np.zeros(n, dtype=np.int64)
        lib().orc_read_eepf(self.h, dptr(f), iptr(c))
        return f, c

    def currents(self):
        je, ji = np.zeros(self.ng), np.zeros(self.ng)
        lib().orc_read_currents(self.h, dptr(je), dptr(ji))
        return je, ji

    def mean_energy(self):
        m = np.zeros(self.ng)
        lib().orc_read_mean_energy(self.h, dptr(m))
        return m

    def reset_diag(self):
        lib().orc_reset_diag(self.h)

    @property
    def n_xt(self) -> int:
        return lib().orc_n_xt(self.h)

    def xt(self, name: str) -> np.ndarray:
        """xt array `name` (one of XT_NAMES) as [n_xt, n_grid]."""
        out = np.zeros((max(self.n_xt, 1), self.ng))
        lib().orc_read_xt(self.h, XT_NAMES.index(name), dptr(out))
        return out[: self.n_xt]

    def xt_steps(self):
        n = max(self.n_xt, 1)
        a, b = np.zeros(n, dtype=np.int64), np.zeros(n, dtype=np.int64)
        lib().orc_xt_steps(self.h, iptr(a), iptr(b))
        return a[: self.n_xt], b[: self.n_xt]

    def ifed(self):
        """(F_powered, F_grounded, counts[2, n_ifed + 1])."""
        nb = self.case.get("n_ifed", 200)
        fp, fg = np.zeros(nb), np.zeros(nb)
        c = np.zeros(2 * (nb + 1), dtype=np.int64)
        lib().orc_read_ifed(self.h, dptr(fp), dptr(fg), iptr(c))
        return fp, fg, c.reshape(2, nb + 1)

    def info(self) -> Dict[str, float]:
        out = np.zeros(len(INFO_NAMES))
        lib().orc_info(self.h, dptr(out))
        return dict(zip(INFO_NAMES, (float(v) for v in out)))

    def constants(self) -> Dict[str, float]:
        a = np.zeros(8)
        lib().orc_constants(self.h, dptr(a))
        keys = ["dx", "dt_i", "factor_w", "factor_e", "factor_i", "gas_n", "sigma_a", "v0"]
        return dict(zip(keys, (float(v) for v in a)))

    def voltage(self, step: int) -> float:
        return lib().orc_voltage(self.h, step)

    def set_voltage(self, v_amp, v_dc: float = 0.0):
        a = np.ascontiguousarray(v_amp, dtype=np.float64)
        if lib().orc_set_voltage(self.h, dptr(a) if a.size else None, a.size, float(v_dc)) != 0:
            raise ValueError("oracle: " + lib().orc_error().decode())

    def nsig_tot(self):
        nb = self._arrs[0].size
        a, b = np.zeros(nb), np.zeros(nb)
        lib().orc_nsig_tot(self.h, dptr(a), dptr(b))
        return a, b

    def null_params(self) -> Dict[str, float]:
        out = np.zeros(4)
        lib().orc_null_params(self.h, dptr(out))
        return {"nu_star_e": out[0], "nu_star_i": out[1], "p_null_e": out[2], "p_null_i": out[3]}

    def energy_bin(self, energy_ev: float) -> int:
        return int(lib().orc_energy_bin(self.h, float(energy_ev)))

    def collide_electron(self, v, idx, r_proc, r_chi, r_eta, r_share):
        vin = np.ascontiguousarray(v, dtype=np.float64)
        vo, ve = np.zeros(3), np.zeros(3)
        an = C.c_int(0)
        proc = lib().orc_collide_electron(self.h, dptr(vin), int(idx), r_proc, r_chi, r_eta,
                                          r_share, dptr(vo), dptr(ve), C.byref(an))
        return proc, vo, ve, an.value

    def collide_ion(self, v, va, idx, r_proc, r_chi, r_eta):
        vin = np.ascontiguousarray(v, dtype=np.float64)
        vain = np.ascontiguousarray(va, dtype=np.float64)
        vo = np.zeros(3)
        proc = lib().orc_collide_ion(self.h, dptr(vin), dptr(vain), int(idx), r_proc, r_chi,
                                     r_eta, dptr(vo))
        return proc, vo


# Free functions ---------------------------------------------------------------

def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def uniform2(seed, uid, step, species, purpose, call):
    o = np.zeros(2)
    lib().orc_uniform2(seed, uid, step, species, purpose, call, dptr(o))
    return o


def deposit(x: np.ndarray, ng: int, inv_dx: float) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    cnt = np.zeros(ng, dtype=np.int64)
    lib().orc_deposit(dptr(x), x.size, ng, inv_dx, iptr(cnt))
    return cnt


def poisson(ng: int, dx: float, rho: np.ndarray, v_left: float) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.zeros(ng)
    lib().orc_poisson(ng, dx, dptr(rho), v_left, dptr(phi))
    return phi


def efield(ng: int, dx: float, phi: np.ndarray, rho: np.ndarray) -> np.ndarray:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    E = np.zeros(ng)
    lib().orc_efield(ng, dx, dptr(phi), dptr(rho), dptr(E))
    return E


def scatter(g, gmag, gnew, f2, cos_chi, sin_chi, eta, w):
    g = np.ascontiguousarray(g, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_scatter(dptr(g), gmag, gnew, f2, cos_chi, sin_chi, eta, dptr(w), dptr(out))
    return out


def child_uid(parent: int, step: int, kind: int) -> int:
    return int(lib().orc_child_uid(parent, step, kind))


def plasma_params(n_e: float, te_ev: float):
    """(Debye length [m], electron plasma frequency [rad/s])."""
    out = np.zeros(2)
    lib().orc_plasma_params(n_e, te_ev, dptr(out))
    return float(out[0]), float(out[1])


def nu_star(nsig: np.ndarray, de_ev: float, mass: float) -> float:
    a = np.ascontiguousarray(nsig, dtype=np.float64)
    return lib().orc_nu_star(dptr(a), a.size, de_ev, mass)
