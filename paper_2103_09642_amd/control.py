"""Outer control loops over RF cycles, the extensions suggested in section 5:

* DC self-bias: at a blocking-capacitor electrode the conduction currents of
  the two charge signs must cancel on time average.  Each window measures,
  at the powered electrode, the ions absorbed plus the secondary electrons
  emitted (positive charge in) against the electrons absorbed, and moves the
  DC offset of the driving voltage by  gain * imbalance * V_ref, with
  imbalance = (N_i + N_see - N_e) / (N_i + N_see + N_e) and V_ref the sum of
  the harmonic amplitudes: too many electrons (a negative imbalance) push the
  bias down, which repels them.
* Power target: each window measures the absorbed power density (space-time
  mean of j.E over both species, the xt measurement) and scales every
  harmonic amplitude by 1 + gain * (P_target / P - 1), clamped to
  [1/clamp, clamp].  Near the target, with P growing like V^2, the error
  shrinks by |1 - 2 gain| per window, so a gain below 1/2 approaches the
  target without overshoot and a gain above 1 oscillates with a growing
  amplitude: the loop needs the low gain the paper asks for.

Both loops are host logic over the C ABI and run many cases at once: every
window advances all active cases together (one batched call), then reads
each case's measurement and sets its next waveform.  A "plant" is anything
with counts(), info(), reset_diag() and set_voltage(v_amp, v_dc); `advance`
advances a list of plants by a number of steps.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Dict, List, Sequence

import numpy as np


@dataclass
class LoopCase:
    """Per-case state of a control loop: the current waveform and history."""
    plant: object
    v_amp: np.ndarray
    v_dc: float = 0.0
    converged: bool = False
    history: List[Dict] = field(default_factory=list)


def _cases(plants, cases: Sequence[Dict]) -> List[LoopCase]:
    out = []
    for p, c in zip(plants, cases):
        amp = np.array([h[0] for h in c.get("harmonics", [])], dtype=np.float64)
        out.append(LoopCase(p, amp, float(c.get("v_dc", 0.0))))
    return out


def electrode_balance(before: Dict[str, int], after: Dict[str, int]):
    """(positive, negative) charges that reached the powered electrode
    between two counter readings: ions absorbed plus secondaries emitted,
    and electrons absorbed."""
    pos = (after["abs_i_pow"] - before["abs_i_pow"]) + (after["see_pow"] - before["see_pow"])
    neg = after["abs_e_pow"] - before["abs_e_pow"]
    return pos, neg


def self_bias(plants, cases: Sequence[Dict], advance: Callable[[List, int], None], window_steps: int,
              gain: float = 0.2, tol: float = 0.02, max_iter: int = 50) -> List[LoopCase]:
    """Iterate the DC offset of each case until the powered electrode's
    charge imbalance over a window is below `tol` (or max_iter windows)."""
    loop = _cases(plants, cases)
    for lc in loop:
        lc.plant.set_voltage(lc.v_amp, lc.v_dc)
    for it in range(max_iter):
        active = [lc for lc in loop if not lc.converged]
        if not active:
            break
        before = [lc.plant.counts() for lc in active]
        advance([lc.plant for lc in active], window_steps)
        for lc, b in zip(active, before):
            pos, neg = electrode_balance(b, lc.plant.counts())
            tot = pos + neg
            imb = (pos - neg) / tot if tot > 0 else 0.0
            lc.history.append({"iter": it, "v_dc": lc.v_dc, "imbalance": imb, "charges": tot})
            if tot > 0 and abs(imb) < tol:
                lc.converged = True
                continue
            v_ref = float(np.abs(lc.v_amp).sum()) or 1.0
            lc.v_dc += gain * imb * v_ref
            lc.plant.set_voltage(lc.v_amp, lc.v_dc)
    return loop


def power_target(plants, cases: Sequence[Dict], advance: Callable[[List, int], None], window_steps: int,
                 target_w_m3: float, gain: float = 0.3, tol: float = 0.02, clamp: float = 1.25,
                 max_iter: int = 50) -> List[LoopCase]:
    """Iterate the harmonic amplitudes of each case until the absorbed power
    density over a window is within `tol` (relative) of the target.  The
    cases need the xt measurement (flag "xt")."""
    if not (target_w_m3 > 0 and 0 < gain and clamp > 1):
        raise ValueError("need target > 0, gain > 0 and clamp > 1")
    loop = _cases(plants, cases)
    for lc in loop:
        lc.plant.set_voltage(lc.v_amp, lc.v_dc)
    for it in range(max_iter):
        active = [lc for lc in loop if not lc.converged]
        if not active:
            break
        for lc in active:
            lc.plant.reset_diag()
        advance([lc.plant for lc in active], window_steps)
        for lc in active:
            inf = lc.plant.info()
            p = inf["power_e"] + inf["power_i"]
            lc.history.append({"iter": it, "v_amp": lc.v_amp.copy(), "power": p})
            if p > 0 and abs(p / target_w_m3 - 1.0) < tol:
                lc.converged = True
                continue
            f = 1.0 + gain * (target_w_m3 / p - 1.0) if p > 0 else clamp
            f = min(max(f, 1.0 / clamp), clamp)
            lc.v_amp = lc.v_amp * f
            lc.plant.set_voltage(lc.v_amp, lc.v_dc)
    return loop


def gpu_advance(ctx):
    """`advance` for library cases of one context: one batched call."""
    def adv(plants, steps):
        ctx.advance_steps(plants, [steps] * len(plants))
    return adv
