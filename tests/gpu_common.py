"""Helpers shared by the GPU tests: build both sides from one case dict and
compare states particle by particle (matched by uid)."""
import sys

import numpy as np
import pytest

STATE_KEYS = ("x", "vx", "vy", "vz")


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_context():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    from paper_2103_09642_amd import edupic
    edupic.load()  # raises if the HIP library is missing: no fallback
    return edupic.Context(0)


def by_uid(st):
    o = np.argsort(st["uid"], kind="stable")
    return {k: v[o] for k, v in st.items()}


def compare_states(a, b, rtol, label="", floors=None):
    """Same uids; every component within rtol relative to its own value, or
    to 1e-3 of the component's largest value (or floors[key]) where that is
    larger; returns the number of bit-exact mismatches."""
    a, b = by_uid(a), by_uid(b)
    assert a["uid"].size == b["uid"].size, f"{label}: {a['uid'].size} vs {b['uid'].size} particles"
    assert np.array_equal(a["uid"], b["uid"]), f"{label}: particle identities differ"
    mism = 0
    for k in STATE_KEYS:
        if a[k].size == 0:
            continue
        scale = max(np.abs(a[k]).max(), 1e-300)
        err = np.abs(a[k] - b[k])
        # relative to the value where the value is large, to the scale otherwise
        floor = max(1e-3 * scale, (floors or {}).get(k, 0.0))
        rel = err / np.maximum(np.abs(b[k]), floor)
        worst = int(np.argmax(rel))
        assert rel[worst] <= rtol, f"{label}: {k}[{worst}] {a[k][worst]!r} vs {b[k][worst]!r} (rel {rel[worst]:.3e})"
        mism += int(np.count_nonzero(a[k] != b[k]))
    return mism


def make_pair(ctx, case, xs, orc):
    g = ctx.create_case(case)
    o = orc.Oracle(case, xs)
    return g, o


def set_both(g, o, st, step):
    for sp, key in ((0, "e"), (1, "i")):
        g.set_state(sp, st[key], step)
        o.set_state(sp, st[key], step)


def poisson_reference(rho, dx, v_left):
    """The grid field of the discrete Poisson equation solved in extended
    (80-bit) precision, for judging FP64 solvers."""
    eps0 = 8.8541878128e-12
    ld = np.longdouble
    ng = rho.size
    d = np.asarray(rho[1:-1], dtype=ld) * (ld(dx) * ld(dx) / ld(eps0))
    S = np.cumsum(d)
    F0 = (ld(v_left) - S.sum()) / ld(ng - 1)
    F = np.concatenate([[F0], F0 + S])
    E = np.empty(ng, dtype=ld)
    E[1:-1] = (F[:-1] + F[1:]) / (2 * ld(dx))
    E[0] = F[0] / ld(dx) - ld(rho[0]) * ld(dx) / (2 * ld(eps0))
    E[-1] = F[-1] / ld(dx) + ld(rho[-1]) * ld(dx) / (2 * ld(eps0))
    return E
