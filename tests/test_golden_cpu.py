"""The stored oracle trajectories (tests/golden/rk4_n256_2000.npz, written by
tests/golden/make_rk4_n256.py from the FP64 oracle) against the oracle as it
stands and against the conservation the projected operator guarantees."""
import os

import numpy as np

import oracle
from paper_2607_00755_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def _gold():
    with np.load(os.path.join(HERE, "golden", "rk4_n256_2000.npz"), allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def test_rk4_fixture_rows_and_conservation():
    """Rows are the documented seeded picks; every stored state keeps the
    number and energy moments of its initial state (App. C projection: at
    most 1e-12 relative drift per step, 2000 steps)."""
    g = _gold()
    assert int(g["steps"]) == 2000
    assert np.array_equal(g["batched_rows"], np.linspace(0, 511, 16).astype(np.int64))
    assert np.array_equal(g["mixed_rows"], np.linspace(0, 4095, 16).astype(np.int64))
    w = inputs.mixed_n256(4096)
    p = w.grid()
    op = oracle.Operator(p)
    for name in ("batched", "mixed"):
        for j, b in enumerate(g[name + "_rows"]):
            m0 = op.moments(w.solves[int(b)].f0(p))
            m1 = g[name + "_moments"][j]
            assert np.all(np.abs(m1[:2] - m0[:2]) <= 2000 * 1e-12 * np.abs(m0[:2])), (name, int(b))
            assert np.array_equal(m1, op.moments(g[name + "_f"][j]))


def test_rk4_fixture_is_what_the_oracle_computes():
    """One stored solve (the last row of the mixed-precision picks) recomputed
    from its seeded input with the oracle."""
    g = _gold()
    w = inputs.mixed_n256(4096)
    p = w.grid()
    op = oracle.Operator(p)
    b = int(g["mixed_rows"][-1])
    s = w.solves[b]
    f0 = s.f0(p)
    dt = 0.1 / (s.lam * op.gamma0(f0))
    assert dt == g["mixed_dt"][-1]
    f = op.rk4(f0, s.lam, dt, 2000)
    ref = g["mixed_f"][-1]
    assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))
