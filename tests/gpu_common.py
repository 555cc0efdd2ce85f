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


def compare_states(a, b, rtol, label=""):
    """Same uids; every component within rtol relative to the component's
    scale (max |value| over the species); returns the number of bit-exact
    mismatches."""
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
        rel = err / np.maximum(np.abs(b[k]), 1e-3 * scale)
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
