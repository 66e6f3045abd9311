"""Write rk4_n256_2000.npz: the oracle's state after 2000 projected RK4 steps
(df/dt = lambda C_proj[f], dt = 0.1 / (lambda Gamma0)) for 16 seeded solves of
the batched N=256 workload (rows spread over 0..511) and 16 of the
mixed-precision workload (rows spread over 0..4095), with the number and
energy moments of each final state.

Every stored value comes from the FP64 oracle (`oracle/`), run on the seeded
inputs of `paper_2607_00755_amd/inputs.py`; nothing is taken from the device
path.  Run from the repository root:

    python tests/golden/make_rk4_n256.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2607_00755_amd import inputs  # noqa: E402

STEPS = 2000
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rk4_n256_2000.npz")


def main():
    oracle.build(force=False)
    w = inputs.mixed_n256(4096)
    p = w.grid()
    f0 = w.f0()
    op = oracle.Operator(p)
    rows = {"batched": np.linspace(0, 511, 16).astype(np.int64),
            "mixed": np.linspace(0, 4095, 16).astype(np.int64)}
    out = {}
    for name, sel in rows.items():
        fin, dts, mom = [], [], []
        for b in sel:
            s = w.solves[int(b)]
            dt = 0.1 / (s.lam * op.gamma0(f0[b]))
            f = op.rk4(f0[b], s.lam, dt, STEPS)
            fin.append(f)
            dts.append(dt)
            mom.append(op.moments(f))
            print(name, int(b), "dt %.6g" % dt, flush=True)
        out[name + "_rows"] = sel
        out[name + "_f"] = np.stack(fin)
        out[name + "_dt"] = np.array(dts)
        out[name + "_moments"] = np.stack(mom)
    out["steps"] = np.array(STEPS)
    np.savez(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
