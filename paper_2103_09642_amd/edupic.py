"""ctypes binding of libedupic.so (include/edupic.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels; PyTorch only
provides the device arena (a uint8 tensor) and the stream.  The binding fails
loudly when the library has not been built -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libedupic.so")

EDP_OK, EDP_EINVAL, EDP_ECAPACITY, EDP_EUNSTABLE, EDP_EHIP, EDP_EARENA, EDP_ESTATE = 0, -1, -2, -3, -4, -5, -6
DIAG_DENSITY, DIAG_EEPF, DIAG_CURRENT, DIAG_MEANE, IONIZ_ANGLE_LITERAL, ALLOW_UNSTABLE = 1, 2, 4, 8, 16, 32
NULL_COLLISION, DIAG_XT, DIAG_IFED = 64, 128, 256
XT_NAMES = ["pot", "efield", "ne", "ni", "je", "ji", "powere", "poweri", "meanee", "meanei", "ioniz"]
INFO_NAMES = ["mean_e", "ne_max", "debye", "dx_debye", "wpe_dt", "pmax_e", "pmax_i", "cfl_ev",
              "power_e", "power_i", "flux_i_pow", "flux_i_gnd", "ei_pow", "ei_gnd", "fail"]
OPT_MODE, OPT_SORT_EVERY, OPT_PROFILE, OPT_GRAPH_STEPS = 1, 2, 5, 6
OPT_POISSON = 8
OPT_PART_WG_PER_CU = 9
OPT_GROUPS = 11
OPT_PART_SKEW = 13
OPT_PRETEST = 14
OPT_SMALL_MAX = 12
POISSON_FLUX, POISSON_THOMAS = 0, 1
MODE_PLAIN, MODE_GRAPH = 0, 1
ELECTRONS, IONS = 0, 1
_FLAG_NAMES = {"density": DIAG_DENSITY, "eepf": DIAG_EEPF, "current": DIAG_CURRENT,
               "meane": DIAG_MEANE, "ioniz_literal": IONIZ_ANGLE_LITERAL,
               "allow_unstable": ALLOW_UNSTABLE, "null_collision": NULL_COLLISION,
               "xt": DIAG_XT, "ifed": DIAG_IFED}


class EdpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"edupic error {code}: {msg}")
        self.code = code


class CaseDesc(C.Structure):
    _fields_ = [("gap_m", C.c_double), ("pressure_pa", C.c_double), ("gas_temp_k", C.c_double),
                ("area_m2", C.c_double), ("n_grid", C.c_int32), ("steps_per_cycle", C.c_int32),
                ("ion_subcycle", C.c_int32), ("n_harm", C.c_int32), ("dt_e", C.c_double),
                ("v_amp", C.c_double * 4), ("freq_hz", C.c_double * 4),
                ("phase_rad", C.c_double * 4), ("weight", C.c_double), ("n_init_e", C.c_int64),
                ("n_init_i", C.c_int64), ("te_init_ev", C.c_double), ("ti_init_k", C.c_double),
                ("cap_e", C.c_int64), ("cap_i", C.c_int64), ("seed", C.c_uint64),
                ("flags", C.c_uint32), ("n_eepf", C.c_int32), ("de_eepf_ev", C.c_double),
                ("n_xt_bin", C.c_int32), ("n_ifed", C.c_int32), ("de_ifed_ev", C.c_double),
                ("gamma_see", C.c_double * 2), ("eta_refl", C.c_double * 2), ("see_te_ev", C.c_double),
                ("v_dc", C.c_double)]


class Xsec(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("de_ev", C.c_double),
                ("e_el", C.POINTER(C.c_double)), ("e_exc", C.POINTER(C.c_double)),
                ("e_ion", C.POINTER(C.c_double)), ("i_iso", C.POINTER(C.c_double)),
                ("i_back", C.POINTER(C.c_double)), ("e_exc_thr_ev", C.c_double),
                ("e_ion_thr_ev", C.c_double), ("w_ioniz_ev", C.c_double)]


class Counts(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "n_e", "n_i", "step", "abs_e_pow", "abs_e_gnd", "abs_i_pow", "abs_i_gnd", "coll_e",
        "coll_i", "ioniz", "anomalies", "dropped", "psteps_e", "psteps_i", "see_pow", "see_gnd", "refl")]

    def as_dict(self) -> Dict[str, int]:
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


# Every symbol of include/edupic.h (checked by the ABI test).
EXPORTS = ["edp_create", "edp_destroy", "edp_set_xsec", "edp_case_bytes", "edp_case_create",
           "edp_case_destroy", "edp_advance", "edp_advance_steps", "edp_sync", "edp_read_counts",
           "edp_read_density", "edp_read_eepf", "edp_read_currents", "edp_read_mean_energy",
           "edp_read_deposit", "edp_read_fields", "edp_get_state", "edp_set_state",
           "edp_set_option", "edp_read_profile", "edp_last_error", "edp_read_xt",
           "edp_read_xt_steps", "edp_read_ifed", "edp_read_info", "edp_reset_diag", "edp_set_voltage",
           "edp_advance_steps_noalloc", "edp_case_resize"]

_lib = None


def load() -> C.CDLL:
    """Load the library (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    try:
        import torch  # noqa: F401  (its libamdhip64 must be the process's HIP runtime)
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    I64P, U64P = C.POINTER(C.c_int64), C.POINTER(C.c_uint64)
    sig = {
        "edp_create": (C.c_int, [C.POINTER(P), C.c_int, P]),
        "edp_destroy": (C.c_int, [P]),
        "edp_set_xsec": (C.c_int, [P, C.POINTER(Xsec)]),
        "edp_case_bytes": (I64, [P, C.POINTER(CaseDesc)]),
        "edp_case_create": (C.c_int, [P, C.POINTER(CaseDesc), P, I64, I64P]),
        "edp_case_destroy": (C.c_int, [P, I64]),
        "edp_case_resize": (C.c_int, [P, I64, I64, I64, P, I64]),
        "edp_advance": (C.c_int, [P, I64P, I32, C.POINTER(I32)]),
        "edp_advance_steps": (C.c_int, [P, I64P, I32, I64P]),
        "edp_advance_steps_noalloc": (C.c_int, [P, I64P, I32, I64P]),
        "edp_sync": (C.c_int, [P]),
        "edp_read_counts": (C.c_int, [P, I64, C.POINTER(Counts)]),
        "edp_read_density": (C.c_int, [P, I64, D, D, I32, I32]),
        "edp_read_eepf": (C.c_int, [P, I64, D, I64P, I32, I32]),
        "edp_read_currents": (C.c_int, [P, I64, D, D, I32, I32]),
        "edp_read_mean_energy": (C.c_int, [P, I64, D, I32, I32]),
        "edp_read_deposit": (C.c_int, [P, I64, I64P, I64P, I32]),
        "edp_read_fields": (C.c_int, [P, I64, D, D, D, I32]),
        "edp_get_state": (C.c_int, [P, I64, I32, D, D, D, D, U64P, I64, I64P]),
        "edp_set_state": (C.c_int, [P, I64, I32, D, D, D, D, U64P, I64, I64]),
        "edp_set_option": (C.c_int, [P, I32, I64]),
        "edp_read_profile": (C.c_int, [P, D, I64P]),
        "edp_last_error": (C.c_char_p, []),
        "edp_read_xt": (C.c_int, [P, I64, I32, D, I64]),
        "edp_read_xt_steps": (C.c_int, [P, I64, I64P, I64P, I32]),
        "edp_read_ifed": (C.c_int, [P, I64, D, D, I64P, I32]),
        "edp_read_info": (C.c_int, [P, I64, D, I32]),
        "edp_reset_diag": (C.c_int, [P, I64]),
        "edp_set_voltage": (C.c_int, [P, I64, D, I32, C.c_double]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


def _chk(code: int):
    if code < 0:
        raise EdpError(code, load().edp_last_error().decode())
    return code


def _d(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _u(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def make_desc(c: Dict) -> CaseDesc:
    d = CaseDesc()
    d.gap_m, d.pressure_pa, d.gas_temp_k, d.area_m2 = c["gap_m"], c["pressure_pa"], c["gas_temp_k"], c["area_m2"]
    d.n_grid, d.steps_per_cycle, d.ion_subcycle = c["n_grid"], c["steps_per_cycle"], c["ion_subcycle"]
    h = c["harmonics"]
    if len(h) > 4:
        raise ValueError("at most 4 harmonics")
    d.n_harm = len(h)
    for k, (v, f, ph) in enumerate(h):
        d.v_amp[k], d.freq_hz[k], d.phase_rad[k] = v, f, ph
    d.dt_e, d.weight = c["dt_e"], c["weight"]
    d.n_init_e, d.n_init_i = c["n_init_e"], c["n_init_i"]
    d.te_init_ev, d.ti_init_k = c["te_init_ev"], c["ti_init_k"]
    d.cap_e, d.cap_i = c.get("cap_e", 0), c.get("cap_i", 0)
    d.seed = c["seed"]
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


class Context:
    """One library context on a device and a torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self._torch = torch
        L = load()
        self.device = device
        torch.cuda.set_device(device)
        # a stream of its own (default priority): hipGraph capture cannot use
        # the legacy default stream
        self.stream = stream if stream is not None else torch.cuda.Stream(device)
        h = C.c_void_p()
        _chk(L.edp_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream)))
        self.h = h
        self._xs_keep = None

    def close(self):
        if getattr(self, "h", None):
            load().edp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_xsec(self, xs: Dict):
        arrs = [np.ascontiguousarray(xs[k], dtype=np.float64) for k in ("e_el", "e_exc", "e_ion", "i_iso", "i_back")]
        x = Xsec()
        x.n_bins, x.de_ev = xs["n_bins"], xs["de_ev"]
        x.e_el, x.e_exc, x.e_ion, x.i_iso, x.i_back = (_d(a) for a in arrs)
        x.e_exc_thr_ev, x.e_ion_thr_ev, x.w_ioniz_ev = xs["e_exc_thr_ev"], xs["e_ion_thr_ev"], xs["w_ioniz_ev"]
        _chk(load().edp_set_xsec(self.h, C.byref(x)))

    def set_option(self, key: int, value: int):
        _chk(load().edp_set_option(self.h, key, value))

    def case_bytes(self, case: Dict) -> int:
        d = make_desc(case)
        return _chk(load().edp_case_bytes(self.h, C.byref(d)))

    def create_case(self, case: Dict) -> "Case":
        return Case(self, case)

    def advance(self, cases: Sequence["Case"], cycles: Sequence[int]):
        n = len(cases)
        ids = (C.c_int64 * n)(*[c.id for c in cases])
        cy = (C.c_int32 * n)(*cycles)
        _chk(load().edp_advance(self.h, ids, n, cy))

    def advance_steps(self, cases: Sequence["Case"], steps: Sequence[int]):
        n = len(cases)
        ids = (C.c_int64 * n)(*[c.id for c in cases])
        st = (C.c_int64 * n)(*steps)
        _chk(load().edp_advance_steps(self.h, ids, n, st))

    def advance_steps_noalloc(self, cases: Sequence["Case"], steps: Sequence[int]):
        """edp_advance_steps_noalloc: the same advance with no device
        allocation (role table in the library's per-device static array)."""
        n = len(cases)
        ids = (C.c_int64 * n)(*[c.id for c in cases])
        st = (C.c_int64 * n)(*steps)
        _chk(load().edp_advance_steps_noalloc(self.h, ids, n, st))

    def sync(self):
        _chk(load().edp_sync(self.h))

    def read_profile(self):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        _chk(load().edp_read_profile(self.h, C.byref(ms), C.byref(n)))
        return ms.value, n.value


class Case:
    """A case and its device arena (a torch uint8 tensor kept alive here)."""

    def __init__(self, ctx: Context, case: Dict):
        self.ctx = ctx
        self.case = case
        self.ng = case["n_grid"]
        d = make_desc(case)
        nbytes = _chk(load().edp_case_bytes(ctx.h, C.byref(d)))
        torch = ctx._torch
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{ctx.device}")
        base = self.arena.data_ptr()
        aligned = (base + 255) // 256 * 256
        out = C.c_int64(0)
        _chk(load().edp_case_create(ctx.h, C.byref(d), C.c_void_p(aligned), nbytes, C.byref(out)))
        self.id = out.value

    def resize(self, cap_e: int = 0, cap_i: int = 0):
        """Move the case into a new arena with other particle capacities (0:
        keep); the run continues unchanged."""
        case = dict(self.case)
        if cap_e:
            case["cap_e"] = cap_e
        if cap_i:
            case["cap_i"] = cap_i
        d = make_desc(case)
        nbytes = _chk(load().edp_case_bytes(self.ctx.h, C.byref(d)))
        torch = self.ctx._torch
        arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        aligned = (arena.data_ptr() + 255) // 256 * 256
        _chk(load().edp_case_resize(self.ctx.h, self.id, int(cap_e), int(cap_i), C.c_void_p(aligned), nbytes))
        self.arena = arena  # the old arena is released here
        self.case = case

    def capacity(self):
        """(cap_e, cap_i) as the library rounds them."""
        def cap(n_init, c):
            v = c if c > 0 else max(2 * n_init, 1 << 18)
            return (v + 255) // 256 * 256
        return cap(self.case["n_init_e"], self.case.get("cap_e", 0)), cap(self.case["n_init_i"], self.case.get("cap_i", 0))

    def destroy(self):
        if self.id:
            _chk(load().edp_case_destroy(self.ctx.h, self.id))
            self.id = 0
            self.arena = None

    def advance(self, cycles: int):
        self.ctx.advance([self], [cycles])

    def advance_steps(self, steps: int):
        self.ctx.advance_steps([self], [steps])

    def counts(self) -> Dict[str, int]:
        """Counters; "overflow" is 1 when the case has exceeded its capacity
        (the library then reports EDP_ECAPACITY with the counters filled)."""
        c = Counts()
        code = load().edp_read_counts(self.ctx.h, self.id, C.byref(c))
        if code != EDP_ECAPACITY:
            _chk(code)
        d = c.as_dict()
        d["overflow"] = int(code == EDP_ECAPACITY)
        return d

    def density(self, reset: bool = False):
        ne, ni = np.zeros(self.ng), np.zeros(self.ng)
        _chk(load().edp_read_density(self.ctx.h, self.id, _d(ne), _d(ni), self.ng, int(reset)))
        return ne, ni

    def eepf(self, reset: bool = False):
        n = self.case["n_eepf"]
        f, c = np.zeros(n), np.zeros(n, dtype=np.int64)
        _chk(load().edp_read_eepf(self.ctx.h, self.id, _d(f), _i(c), n, int(reset)))
        return f, c

    def currents(self, reset: bool = False):
        je, ji = np.zeros(self.ng), np.zeros(self.ng)
        _chk(load().edp_read_currents(self.ctx.h, self.id, _d(je), _d(ji), self.ng, int(reset)))
        return je, ji

    def mean_energy(self, reset: bool = False):
        m = np.zeros(self.ng)
        _chk(load().edp_read_mean_energy(self.ctx.h, self.id, _d(m), self.ng, int(reset)))
        return m

    @property
    def n_xt(self) -> int:
        if "xt" not in self.case.get("flags", []):
            return 0
        return self.case["steps_per_cycle"] // self.case.get("n_xt_bin", 20)

    def xt(self, name: str) -> np.ndarray:
        """xt array `name` (one of XT_NAMES) as [n_xt, n_grid]."""
        out = np.zeros((self.n_xt, self.ng))
        _chk(load().edp_read_xt(self.ctx.h, self.id, XT_NAMES.index(name), _d(out), out.size))
        return out

    def xt_steps(self):
        a, b = np.zeros(self.n_xt, dtype=np.int64), np.zeros(self.n_xt, dtype=np.int64)
        _chk(load().edp_read_xt_steps(self.ctx.h, self.id, _i(a), _i(b), self.n_xt))
        return a, b

    def ifed(self):
        """(F_powered, F_grounded, counts[2, n_ifed + 1])."""
        nb = self.case.get("n_ifed", 200)
        fp, fg = np.zeros(nb), np.zeros(nb)
        c = np.zeros(2 * (nb + 1), dtype=np.int64)
        _chk(load().edp_read_ifed(self.ctx.h, self.id, _d(fp), _d(fg), _i(c), nb))
        return fp, fg, c.reshape(2, nb + 1)

    def info(self) -> Dict[str, float]:
        out = np.zeros(len(INFO_NAMES))
        _chk(load().edp_read_info(self.ctx.h, self.id, _d(out), out.size))
        return dict(zip(INFO_NAMES, (float(v) for v in out)))

    def reset_diag(self):
        _chk(load().edp_reset_diag(self.ctx.h, self.id))

    def set_voltage(self, v_amp, v_dc: float = 0.0):
        """New harmonic amplitudes (one per harmonic of the case) and DC
        offset, effective from the next advance."""
        a = np.ascontiguousarray(v_amp, dtype=np.float64)
        _chk(load().edp_set_voltage(self.ctx.h, self.id, _d(a) if a.size else None, a.size, float(v_dc)))

    def deposit(self):
        a, b = np.zeros(self.ng, dtype=np.int64), np.zeros(self.ng, dtype=np.int64)
        _chk(load().edp_read_deposit(self.ctx.h, self.id, _i(a), _i(b), self.ng))
        return a, b

    def fields(self):
        rho, phi, E = (np.zeros(self.ng) for _ in range(3))
        _chk(load().edp_read_fields(self.ctx.h, self.id, _d(rho), _d(phi), _d(E), self.ng))
        return rho, phi, E

    def get_state(self, species: int) -> Dict[str, np.ndarray]:
        L = load()
        n = C.c_int64(0)
        _chk(L.edp_get_state(self.ctx.h, self.id, species, None, None, None, None, None, 0, C.byref(n)))
        m = n.value
        out = {k: np.empty(m) for k in ("x", "vx", "vy", "vz")}
        out["uid"] = np.empty(m, dtype=np.uint64)
        _chk(L.edp_get_state(self.ctx.h, self.id, species, _d(out["x"]), _d(out["vx"]), _d(out["vy"]),
                             _d(out["vz"]), _u(out["uid"]), m, C.byref(n)))
        return out

    def set_state(self, species: int, st: Dict[str, np.ndarray], step: int):
        a = {k: np.ascontiguousarray(st[k], dtype=np.float64) for k in ("x", "vx", "vy", "vz")}
        u = np.ascontiguousarray(st["uid"], dtype=np.uint64)
        _chk(load().edp_set_state(self.ctx.h, self.id, species, _d(a["x"]), _d(a["vx"]), _d(a["vy"]),
                                  _d(a["vz"]), _u(u), a["x"].size, step))
